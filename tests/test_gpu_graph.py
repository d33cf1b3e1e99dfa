"""GPU checks of graph-replayed shootings and gradients (GS_FLAG_GRAPH).

A call with GS_FLAG_GRAPH captures its kernel sequence once and replays it on
later calls with the same arguments; the kernels and their arguments are
those of the call without the flag, so every replay must reproduce the eager
result bit for bit.  The replays are interleaved with other eager calls that
share the workspace (so the per-call table upload is exercised) and with new
values written into the same input buffers.  One case is also held to the
FP64 oracle at the single-set bars (rel-L2 1e-5 on q(1), p(1), 1e-6 on H).
"""
import ctypes
import time

import numpy as np
import pytest
import torch

from helpers import rel_l2
from paper_1907_04834_amd import gs
from paper_1907_04834_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _say(msg):
    print(msg, flush=True)


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b) if x is not None)


def _graph_params(prm):
    g = gs.Params.from_buffer_copy(prm)
    g.flags |= gs.GS_FLAG_GRAPH
    return g


@pytest.mark.parametrize("method", [gs.GS_EXACT, gs.GS_BH])
def test_graph_single_set_replays_equal_eager(method):
    a, b = W.ellipsoid_20k(seed=41, n=3000), W.ellipsoid_20k(seed=42, n=3000)
    prm = gs.params(0.05, nt=8, theta=0.5, leaf_cap=8)
    gprm = _graph_params(prm)
    q0, p0 = _t(a.q0), _t(a.p0)
    ws = gs._workspace(3000, prm, method, gs.GS_OP_SHOOT, q0.device)
    out = (torch.empty_like(q0), torch.empty_like(q0),
           torch.zeros(prm.nt + 1, dtype=torch.float64, device=DEV))
    _say(f"graph single set method={method} n=3000 nt=8")
    ref_a = gs.gs_shoot(q0, p0, prm, method, ws=ws)
    for rep in range(4):
        got = gs.gs_shoot(q0, p0, gprm, method, ws=ws, out=out)
        torch.cuda.synchronize()
        assert _same(got, ref_a), f"replay {rep} differs from the eager call"
        other = gs.gs_shoot(_t(b.q0), _t(b.p0), prm, method, ws=ws)  # same workspace
        torch.cuda.synchronize()
        assert other[0].shape == q0.shape
    # new values in the captured input buffers
    q0.copy_(_t(b.q0))
    p0.copy_(_t(b.p0))
    ref_b = gs.gs_shoot(q0, p0, prm, method, ws=ws)
    for rep in range(2):
        got = gs.gs_shoot(q0, p0, gprm, method, ws=ws, out=out)
        torch.cuda.synchronize()
        assert _same(got, ref_b), f"replay {rep} on new inputs differs from the eager call"


@pytest.mark.parametrize("method", [gs.GS_EXACT, gs.GS_BH])
def test_graph_batch_replays_equal_eager_and_oracle(oracle, method):
    sizes = [900, 1, 0, 1700, 130]
    subs = [W.ellipsoid_20k(seed=60 + k, n=n) if n else
            W.Workload("empty", np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                       0.05, 40, "f32") for k, n in enumerate(sizes)]
    q, p, off = W.stack(subs)
    sigma, nt, theta, leaf_cap = 0.05, 6, 0.5, 4
    prm = gs.params(sigma, nt=nt, theta=theta, leaf_cap=leaf_cap)
    gprm = _graph_params(prm)
    qd, pd = _t(q), _t(p)
    _say(f"graph batch method={method} sizes={sizes}")
    ref = gs.gs_shoot_batch(qd, pd, off, prm, method, return_ws=True)
    ws = ref[3]
    out = (torch.empty_like(qd), torch.empty_like(qd),
           torch.zeros(len(sizes), nt + 1, dtype=torch.float64, device=DEV))
    for rep in range(4):
        got = gs.gs_shoot_batch(qd, pd, off, gprm, method, ws=ws, out=out)
        torch.cuda.synchronize()
        assert _same(got, ref[:3]), f"replay {rep} differs from the eager call"
        gs.gs_shoot_batch(qd, pd, off, prm, method, ws=ws)  # eager work in between
        torch.cuda.synchronize()
    q1, p1, H = _np(out[0]), _np(out[1]), _np(out[2])
    kind = "exact" if method == gs.GS_EXACT else "bh"
    for s, w in enumerate(subs):
        lo, hi = off[s], off[s + 1]
        if hi == lo:
            assert np.all(H[s] == 0.0)
            continue
        qo, po, Ho = oracle.shoot(w.q0.astype(np.float64), w.p0.astype(np.float64), sigma, nt,
                                  method=kind, theta=theta, leaf_cap=leaf_cap)
        eq, ep = rel_l2(q1[lo:hi], qo), rel_l2(p1[lo:hi], po)
        eh = float(np.max(np.abs(H[s] - Ho)) / np.max(np.abs(Ho)))
        _say(f"  set {s} n={hi - lo}: q1 {eq:.2e} p1 {ep:.2e} H {eh:.2e}")
        assert eq < 1e-5 and ep < 1e-5 and eh < 1e-6


@pytest.mark.parametrize("method", [gs.GS_EXACT, gs.GS_BH])
def test_graph_replay_time_small_problem(method):
    """Reports eager vs replayed call time on a launch-bound problem (2000
    points, 40 steps); the replay must not be slower than eager by more than
    timing noise."""
    w = W.ellipsoid_20k(seed=5, n=2000)
    prm = gs.params(0.05, nt=40, theta=0.5, leaf_cap=16)
    gprm = _graph_params(prm)
    q0, p0 = _t(w.q0), _t(w.p0)
    ws = gs._workspace(2000, prm, method, gs.GS_OP_SHOOT, q0.device)
    out = (torch.empty_like(q0), torch.empty_like(q0),
           torch.zeros(prm.nt + 1, dtype=torch.float64, device=DEV))

    def per_call(p, reps=20):
        gs.gs_shoot(q0, p0, p, method, ws=ws, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            gs.gs_shoot(q0, p0, p, method, ws=ws, out=out)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    eager, graph = per_call(prm), per_call(gprm)
    _say(f"n=2000 nt=40 method={method}: eager {eager:.3f} ms, graph {graph:.3f} ms per call")
    assert graph < 1.25 * eager + 0.05


@pytest.mark.parametrize("method", [gs.GS_EXACT, gs.GS_BH])
def test_graph_gradients_replay_equal_eager(method):
    """Graph-replayed objective and gradient (single set and batch) equal the
    eager calls bit for bit, with eager work on the same workspace between
    replays."""
    a = W.adjoint_50k(seed=7, n=3000)
    b = W.adjoint_50k(seed=8, n=3000)
    prm = gs.params(a.sigma, nt=6, theta=0.5, leaf_cap=8)
    gprm = _graph_params(prm)
    q0, p0, y = _t(a.q0), _t(a.p0), _t(a.extra["target"])
    nb = gs.lib().gs_adjoint_workspace_bytes(3000, ctypes.byref(prm), method, 2)
    ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
    out = (torch.zeros(1, dtype=torch.float64, device=DEV), torch.empty_like(q0))
    _say(f"graph gradient method={method} n=3000 nt=6")
    ref = gs.gs_shoot_adjoint(q0, p0, y, prm, method, 0.01, 2, ws=ws)
    for rep in range(3):
        got = gs.gs_shoot_adjoint(q0, p0, y, gprm, method, 0.01, 2, ws=ws, out=out)
        torch.cuda.synchronize()
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), rep
        gs.gs_shoot_adjoint(_t(b.q0), _t(b.p0), _t(b.extra["target"]), prm, method, 0.01, 2,
                            ws=ws)
        torch.cuda.synchronize()
    # a batch of two ragged sets
    q = np.concatenate([a.q0, b.q0[:1700]])
    p = np.concatenate([a.p0, b.p0[:1700]])
    yy = np.concatenate([a.extra["target"], b.extra["target"][:1700]])
    off = [0, 3000, 4700]
    qd, pd, yd = _t(q), _t(p), _t(yy)
    offs = (ctypes.c_int64 * 3)(*off)
    wsb = torch.empty(gs.lib().gs_adjoint_batch_workspace_bytes(offs, 2, ctypes.byref(prm),
                                                                method, 2),
                      dtype=torch.uint8, device=DEV)
    refb = gs.gs_shoot_adjoint_batch(qd, pd, yd, off, prm, method, 0.01, 2, ws=wsb)
    outb = (torch.zeros(2, dtype=torch.float64, device=DEV), torch.empty_like(qd))
    for rep in range(3):
        got = gs.gs_shoot_adjoint_batch(qd, pd, yd, off, gprm, method, 0.01, 2, ws=wsb,
                                        out=outb)
        torch.cuda.synchronize()
        assert torch.equal(got[0], refb[0]) and torch.equal(got[1], refb[1]), rep
