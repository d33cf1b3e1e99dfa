"""Translated point sets: the method depends only on differences q_i - q_j
(Sec. 2.1, eq. 1 and eq. 3), so the GPU's accuracy must not depend on where a
set lies.  The FP32 kernels work relative to each set's FP64 box centre; these
tests hold translated inputs to the same bars as the sets near the origin.

* 20k ellipsoid moved by (100, -50, 30): the oracle runs on the very FP32
  inputs the GPU gets (right-hand side, shooting and gradient, exact and
  Barnes-Hut).  q(1) is compared by rel-L2 as everywhere; its displacement
  q(1) - q(0) is reported too, but an FP32 output at |q| ~ 100 carries a
  rounding of ulp(100) / 2 = 3.8e-6 per coordinate that no kernel can avoid.
* 200k ellipsoids moved by 10: the right-hand sides against the oracle
  (sampled exact rows; the full Barnes-Hut RHS with its counters), and the
  shootings against the GPU's own shooting of the untranslated set, built so
  that the two sets are exact translates of each other in FP32 (the
  untranslated shooting is itself checked against the stored oracle shooting
  in test_gpu_golden.py).
"""
import numpy as np
import pytest
import torch

from helpers import rel_l2
from paper_1907_04834_amd import gs
from paper_1907_04834_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SHIFT20 = np.array([100.0, -50.0, 30.0])


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _say(msg):
    print(msg, flush=True)


def _shifted(q, s):
    return (q.astype(np.float64) + s).astype(np.float32)


_CACHE = {}


def _e20(oracle):
    """The shifted 20k ellipsoid and the oracle's exact shooting of it."""
    if "w" not in _CACHE:
        w = W.ellipsoid_20k()
        qs = _shifted(w.q0, SHIFT20)
        _CACHE["w"] = (w, qs)
        _CACHE["exact"] = oracle.shoot(qs.astype(np.float64), w.p0.astype(np.float64), w.sigma,
                                       w.nt)
    return _CACHE["w"] + (_CACHE["exact"],)


def test_rhs_translated_20k(oracle):
    w, qs, _ = _e20(oracle)
    q64, p64 = qs.astype(np.float64), w.p0.astype(np.float64)
    _say("translated 20k: exact RHS")
    dq, dp = gs.gs_rhs_exact(_t(qs), _t(w.p0), gs.params(w.sigma))
    v, a = oracle.rhs_exact(q64, p64, w.sigma)
    ev, ea = rel_l2(_np(dq), v), rel_l2(_np(dp), a)
    _say(f"  exact rel-L2 v {ev:.3e} a {ea:.3e}")
    assert ev < 1e-5 and ea < 1e-5
    _say("translated 20k: Barnes-Hut RHS")
    prm = gs.params(w.sigma, theta=0.5, leaf_cap=4)
    dq, dp, ws = gs.gs_rhs_bh(_t(qs), _t(w.p0), prm, return_ws=True)
    cnt, st = gs.gs_bh_counters(ws), gs.gs_get_status(ws)
    v, a, oc = oracle.rhs_bh(q64, p64, w.sigma, 0.5, leaf_cap=4)
    ev, ea = rel_l2(_np(dq), v), rel_l2(_np(dp), a)
    _say(f"  bh rel-L2 v {ev:.3e} a {ea:.3e} gpu {cnt} oracle {oc}")
    assert st == 0 and cnt["pairs"] == oc["pairs"] and cnt["monopoles"] == oc["monopoles"]
    assert ev < 1e-5 and ea < 1e-5


def test_exact_shooting_translated_20k(oracle):
    w, qs, (oq, op, oH) = _e20(oracle)
    _say("translated 20k: exact shooting")
    q1, p1, H = gs.gs_shoot(_t(qs), _t(w.p0), gs.params(w.sigma, nt=w.nt))
    torch.cuda.synchronize()
    eq, ep = rel_l2(_np(q1), oq), rel_l2(_np(p1), op)
    ed = rel_l2(_np(q1) - qs, oq - qs)
    eh = np.abs(H.cpu().numpy() - oH).max() / np.abs(oH).max()
    _say(f"  rel-L2 q1 {eq:.3e} p1 {ep:.3e} H {eh:.3e} (displacement {ed:.3e})")
    assert eq < 1e-5 and ep < 1e-5 and eh < 1e-6


def test_bh_shooting_translated_20k(oracle):
    """Bars of the untranslated test (test_gpu_bh.py): q(1), p(1) within
    max(1e-5, 0.1 eps_theta) of the oracle's Barnes-Hut shooting, H within
    max(1e-5, 0.1 eps_H, 2 delta_H)."""
    w, qs, (eq_, ep_, eH) = _e20(oracle)
    theta = 0.5
    _say("translated 20k: Barnes-Hut shooting")
    prm = gs.params(w.sigma, nt=w.nt, theta=theta, leaf_cap=4)
    q1, p1, H = gs.gs_shoot(_t(qs), _t(w.p0), prm, gs.GS_BH)
    torch.cuda.synchronize()
    q64, p64 = qs.astype(np.float64), w.p0.astype(np.float64)
    bq, bp, bH = oracle.shoot(q64, p64, w.sigma, w.nt, method="bh", theta=theta, leaf_cap=4)
    rng = np.random.default_rng(5)
    away = np.where(rng.random(qs.shape) < 0.5, np.inf, -np.inf).astype(np.float32)
    _, _, dH = oracle.shoot(np.nextafter(qs, away).astype(np.float64), p64, w.sigma, w.nt,
                            method="bh", theta=theta, leaf_cap=4)
    eps_q, eps_p = rel_l2(bq, eq_), rel_l2(bp, ep_)
    gq, gp = rel_l2(_np(q1), bq), rel_l2(_np(p1), bp)
    eps_h = np.abs(bH - eH).max() / np.abs(eH).max()
    delta_h = np.abs(dH - bH).max() / np.abs(bH).max()
    gh = np.abs(H.cpu().numpy() - bH).max() / np.abs(bH).max()
    _say(f"  eps q {eps_q:.3e} p {eps_p:.3e} | gpu-vs-bh q {gq:.3e} p {gp:.3e} | "
         f"H eps {eps_h:.3e} delta {delta_h:.3e} gpu {gh:.3e}")
    assert gq <= max(1e-5, 0.1 * eps_q) and gp <= max(1e-5, 0.1 * eps_p)
    assert gh <= max(1e-5, 0.1 * eps_h, 2.0 * delta_h)


@pytest.mark.parametrize("method", ["exact", "bh"])
def test_gradient_translated(oracle, method):
    """Objective and gradient of a translated template (and target) at the
    untranslated bars: 1e-6 / 1e-5 exact, 1e-5 / 1e-5 Barnes-Hut."""
    w = W.adjoint_50k(n=2000)
    qs = _shifted(w.q0, SHIFT20)
    ys = _shifted(w.extra["target"], SHIFT20)
    nt, lam, ck, theta, lc = 10, 0.01, 3, 0.5, 4
    m = gs.GS_EXACT if method == "exact" else gs.GS_BH
    prm = gs.params(w.sigma, nt=nt, theta=theta, leaf_cap=lc)
    _say(f"translated gradient {method}")
    e, g = gs.gs_shoot_adjoint(_t(qs), _t(w.p0), _t(ys), prm, m, lam, ck)
    torch.cuda.synchronize()
    oe, og = oracle.objective_grad(qs.astype(np.float64), w.p0.astype(np.float64),
                                   ys.astype(np.float64), w.sigma, nt, lam, method=method,
                                   theta=theta, leaf_cap=lc)
    ee, eg = abs(float(e) - oe) / abs(oe), rel_l2(_np(g), og)
    _say(f"  objective {ee:.3e} gradient {eg:.3e}")
    assert ee <= (1e-6 if method == "exact" else 1e-5) and eg < 1e-5


# ------------------------------------------------------------------ 200k + 10
def _e200():
    if "w200" not in _CACHE:
        w = W.ellipsoids_200k()
        qs = _shifted(w.q0, 10.0)
        qb = (qs.astype(np.float64) - 10.0).astype(np.float32)  # exact (Sterbenz)
        assert np.array_equal((qb.astype(np.float64) + 10.0).astype(np.float32), qs)
        _CACHE["w200"] = (w, qs, qb)
    return _CACHE["w200"]


def test_rhs_translated_200k(oracle):
    w, qs, _ = _e200()
    q64, p64 = qs.astype(np.float64), w.p0.astype(np.float64)
    _say("translated 200k: exact RHS (sampled rows)")
    dq, dp = gs.gs_rhs_exact(_t(qs), _t(w.p0), gs.params(w.sigma))
    idx = np.sort(np.random.default_rng(7).choice(w.n, 1024, replace=False))
    v, a = oracle.rhs_exact_rows(idx, q64, p64, w.sigma)
    ev, ea = rel_l2(_np(dq)[idx], v), rel_l2(_np(dp)[idx], a)
    _say(f"  exact rel-L2 v {ev:.3e} a {ea:.3e}")
    assert ev < 1e-5 and ea < 1e-5
    _say("translated 200k: Barnes-Hut RHS")
    prm = gs.params(w.sigma, theta=0.5, leaf_cap=16)
    dq, dp, ws = gs.gs_rhs_bh(_t(qs), _t(w.p0), prm, return_ws=True)
    cnt, st = gs.gs_bh_counters(ws), gs.gs_get_status(ws)
    v, a, oc = oracle.rhs_bh(q64, p64, w.sigma, 0.5, leaf_cap=16)
    ev, ea = rel_l2(_np(dq), v), rel_l2(_np(dp), a)
    _say(f"  bh rel-L2 v {ev:.3e} a {ea:.3e} gpu {cnt} oracle {oc}")
    assert st == 0 and cnt["pairs"] == oc["pairs"] and cnt["monopoles"] == oc["monopoles"]
    assert ev < 1e-5 and ea < 1e-5


@pytest.mark.parametrize("method", ["exact", "bh"])
def test_shooting_translated_200k_equals_untranslated(method):
    """The shooting of the set moved by 10 equals the shooting of the set
    itself moved by 10: p(1) and H(t) to 1e-7 (the two runs differ only in
    the FP64 rounding of the state at magnitude 10 rather than 1, which can
    move an FP32 copy of a position by one ulp now and then), q(1) to the
    1e-5 bar (the FP32 output at magnitude 10 rounds to 4.8e-7)."""
    w, qs, qb = _e200()
    m = gs.GS_EXACT if method == "exact" else gs.GS_BH
    prm = gs.params(w.sigma, nt=w.nt, theta=0.5, leaf_cap=64)
    _say(f"translated 200k shooting {method}")
    q1s, p1s, Hs = gs.gs_shoot(_t(qs), _t(w.p0), prm, m)
    q1b, p1b, Hb = gs.gs_shoot(_t(qb), _t(w.p0), prm, m)
    torch.cuda.synchronize()
    eq = rel_l2(_np(q1s) - 10.0, _np(q1b))
    ep = rel_l2(_np(p1s), _np(p1b))
    eh = np.abs(_np(Hs) - _np(Hb)).max() / np.abs(_np(Hb)).max()
    _say(f"  q1 {eq:.3e} p1 {ep:.3e} H {eh:.3e}")
    assert eq < 1e-5 and ep < 1e-7 and eh < 1e-7
