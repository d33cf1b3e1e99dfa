"""GPU backward stage (discrete adjoint of the Euler flow) against the FP64
oracle, finite differences and its own invariances.

Tolerances: the GPU adjoint uses FP32 pair arithmetic with FP64 sums and an
FP64 state (the gradient computation keeps FP64): gradient rel-L2 1e-5 against the oracle's
exact adjoint; directional derivatives within 1e-4 relative of central
differences (h = 1e-4) of the FP64 GPU forward; the Barnes-Hut backward stage
within 1e-5 of the oracle's Barnes-Hut gradient (measured ~5e-8; the
oracle's own Barnes-Hut vs exact gradient difference eps is printed beside
it).
"""
import numpy as np
import pytest
import torch

import helpers as H
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


def _adj(w, n_steps, lam, ckpt, method=gs.GS_EXACT, theta=0.5, leaf_cap=1):
    y = w.extra["target"]
    prm = gs.params(w.sigma, nt=n_steps, theta=theta, leaf_cap=leaf_cap)
    e, g = gs.gs_shoot_adjoint(_t(w.q0), _t(w.p0), _t(y), prm, method, lam, ckpt)
    torch.cuda.synchronize()
    return float(e), _np(g)


@pytest.mark.parametrize("n,nt,ckpt", [(1, 4, 2), (700, 6, 4), (2000, 10, 3)])
def test_exact_adjoint_matches_oracle(oracle, n, nt, ckpt):
    w = W.adjoint_50k(n=n)
    _say(f"adjoint exact n={n} nt={nt} ckpt={ckpt}")
    e, g = _adj(w, nt, 0.01, ckpt)
    q, p, y = (x.astype(np.float64) for x in (w.q0, w.p0, w.extra["target"]))
    oe, og = oracle.objective_grad(q, p, y, w.sigma, nt, 0.01)
    _say(f"  objective rel {abs(e - oe) / abs(oe):.3e}  grad rel-L2 {rel_l2(g, og):.3e}")
    assert abs(e - oe) <= 1e-6 * abs(oe)
    assert rel_l2(g, og) < 1e-5


def test_checkpoint_interval_does_not_change_the_gradient():
    """Recomputed segments repeat the first forward pass bit for bit."""
    w = W.adjoint_50k(n=3000)
    ref = _adj(w, 12, 0.01, 1)
    for ck in (2, 5, 12, 50):
        e, g = _adj(w, 12, 0.01, ck)
        assert e == ref[0] and np.array_equal(g, ref[1]), ck


def test_adjoint_finite_differences_50k():
    """Template of 50k points, 40 steps, lambda 0.01, checkpoints every 8:
    central differences of the FP64 GPU forward along 32 random directions."""
    w = W.adjoint_50k()
    n, nt, lam = w.n, w.nt, w.extra["lam"]
    _say("adjoint 50k: gradient")
    e, g = _adj(w, nt, lam, w.extra["ckpt"])
    q0 = _t(w.q0.astype(np.float64))
    y = w.extra["target"].astype(np.float64)
    prm = gs.params(w.sigma, nt=nt)

    def objective(p):
        q1, _, H = gs.gs_shoot_f64(q0, _t(p), prm)
        torch.cuda.synchronize()
        return float(((_np(q1) - y) ** 2).sum() / n + lam * float(H[0]))

    p0 = w.p0.astype(np.float64)
    e64 = objective(p0)
    _say(f"  objective fp32-pairs {e:.10e} fp64 {e64:.10e}")
    assert abs(e - e64) <= 1e-6 * abs(e64)
    h = 1e-4
    worst = 0.0
    for k, u in enumerate(W.directions(42, n, 32)):
        fd = (objective(p0 + h * u) - objective(p0 - h * u)) / (2 * h)
        an = float((g * u).sum())
        worst = max(worst, abs(an - fd) / abs(fd))
        if k % 8 == 0:
            _say(f"  dir {k}: adjoint {an:.8e} fd {fd:.8e}")
    _say(f"  worst relative difference {worst:.3e}")
    assert worst <= 1e-4


def test_bh_adjoint(oracle):
    w = W.adjoint_50k(n=1500)
    nt, lam = 6, 0.01
    q, p, y = (x.astype(np.float64) for x in (w.q0, w.p0, w.extra["target"]))
    # theta = 0: the tree backward stage is the exact adjoint
    e0, g0 = _adj(w, nt, lam, 3, gs.GS_BH, theta=0.0, leaf_cap=4)
    ex, gx = _adj(w, nt, lam, 3)
    assert rel_l2(g0, gx) < 1e-5 and abs(e0 - ex) <= 1e-6 * abs(ex)
    for theta in (0.5, np.inf):
        e, g = _adj(w, nt, lam, 3, gs.GS_BH, theta=theta, leaf_cap=4)
        be, bg = oracle.objective_grad(q, p, y, w.sigma, nt, lam, method="bh", theta=theta,
                                       leaf_cap=4)
        xe, xg = oracle.objective_grad(q, p, y, w.sigma, nt, lam)
        eps = rel_l2(bg, xg)
        _say(f"  bh theta={theta}: eps {eps:.3e} gpu-vs-bh {rel_l2(g, bg):.3e} "
             f"objective {abs(e - be) / abs(be):.3e}")
        assert rel_l2(g, bg) <= 1e-5
        assert abs(e - be) <= 1e-5 * abs(be)


@pytest.mark.parametrize("theta", [0.5, np.inf])
def test_bh_adjoint_deepest_tree(oracle, theta):
    """One step from a set whose tree is 21 levels deep (leaf_cap 1): the
    backward decide phase's level walk and depth-first stacks at their
    deepest.  One step only: every decision is then taken on the FP32 input
    itself (a later state would carry the FP32 rounding of the trajectory,
    and on this set a one-ulp change of q0 moves the Barnes-Hut gradient of
    three steps by 5e-3)."""
    q, p = H.deepest_set()
    y = q + 0.01 * np.sin(3.0 * q[:, [1, 2, 0]])
    prm = gs.params(0.02, nt=1, theta=theta, leaf_cap=1)
    e, g = gs.gs_shoot_adjoint(_t(q), _t(p), _t(y.astype(np.float32)), prm, gs.GS_BH, 0.01, 1)
    torch.cuda.synchronize()
    e, g = float(e), _np(g)
    q64, p64, y64 = (x.astype(np.float64) for x in (q, p, y.astype(np.float32)))
    be, bg = oracle.objective_grad(q64, p64, y64, 0.02, 1, 0.01, method="bh", theta=theta,
                                   leaf_cap=1)
    _, xg = oracle.objective_grad(q64, p64, y64, 0.02, 1, 0.01)
    _say(f"  deepest tree theta={theta}: bh vs exact {rel_l2(bg, xg):.3e} "
         f"gpu vs bh {rel_l2(g, bg):.3e}")
    assert rel_l2(g, bg) <= 1e-5
    assert abs(e - be) <= 1e-5 * abs(be)


def test_bh_adjoint_long_leaf_lists(oracle):
    """Single-point leaves on a dense set: a group's list of leaves to sum
    exactly outgrows its segment, and the rest is summed in the decide
    phase; the gradient must still match the oracle's Barnes-Hut gradient."""
    w = W.adjoint_50k(n=20000)
    nt, lam = 2, 0.01
    q, p, y = (x.astype(np.float64) for x in (w.q0, w.p0, w.extra["target"]))
    e, g = _adj(w, nt, lam, 1, gs.GS_BH, theta=0.5, leaf_cap=1)
    be, bg = oracle.objective_grad(q, p, y, w.sigma, nt, lam, method="bh", theta=0.5, leaf_cap=1)
    _, xg = oracle.objective_grad(q, p, y, w.sigma, nt, lam)
    eps = rel_l2(bg, xg)
    _say(f"  bh leaf_cap 1, n=20000: eps {eps:.3e} gpu-vs-bh {rel_l2(g, bg):.3e} "
         f"objective {abs(e - be) / abs(be):.3e}")
    assert rel_l2(g, bg) <= 1e-5
    assert abs(e - be) <= 1e-5 * abs(be)


def test_autograd_function():
    w = W.adjoint_50k(n=800)
    p0 = _t(w.p0).requires_grad_(True)
    loss = gs.shoot_loss(p0, _t(w.q0), _t(w.extra["target"]), w.sigma, nt=5)
    (g,) = torch.autograd.grad(2.0 * loss, (p0,))
    e, gr = _adj(w, 5, 0.01, 8)
    assert abs(float(loss) - e) == 0.0
    np.testing.assert_allclose(_np(g), 2.0 * gr, rtol=0, atol=0)


@pytest.mark.parametrize("method", ["exact", "bh"])
def test_lbfgs_registration_recovers_the_target(method):
    """L-BFGS over p0 driven by the adjoint gradient (the registration of
    Sec. 2.1): starting from p0 = 0, the objective falls by orders of
    magnitude and the shot template lands on the target."""
    from paper_1907_04834_amd import register
    from paper_1907_04834_amd import workloads as W
    w = W.ellipsoid_20k(seed=21, n=3000)
    q0 = torch.from_numpy(w.q0).to(DEV)
    rng = np.random.default_rng(5)
    pstar = W.bump_field(rng, (w.q0.astype(np.float64) + 1.0) / 2.0, m=16, width=0.15,
                         amp=20.0 / w.n)
    pstar = torch.from_numpy(pstar.astype(np.float32)).to(DEV)
    prm = gs.params(0.05, nt=20, theta=0.5, leaf_cap=16)
    target, _, _ = gs.gs_shoot(q0, pstar, prm, gs.GS_EXACT)
    p_opt, hist = register.register(q0, target, 0.05, nt=20, lam=1e-5, method=method,
                                    max_iter=40)
    q1, _, _ = gs.gs_shoot(q0, p_opt, prm, gs.GS_EXACT if method == "exact" else gs.GS_BH)
    err0 = float(torch.sqrt(((q0 - target) ** 2).sum(1).mean()))
    err = float(torch.sqrt(((q1 - target) ** 2).sum(1).mean()))
    print(f"lbfgs {method}: E {hist[0]:.3e} -> {min(hist):.3e} in {len(hist)} evaluations; "
          f"rms distance to target {err0:.3e} -> {err:.3e}", flush=True)
    assert min(hist) < 1e-2 * hist[0]
    assert err < 0.1 * err0
