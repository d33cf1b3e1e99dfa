"""GPU parity of the batched entry points (independent point sets evaluated in
shared launches).

Every set of a batch must come out as the same set evaluated alone: against
the FP64 oracle per set with the single-set bars (rel-L2 1e-5 for one RHS,
1e-5 for q(1), p(1), 1e-6 for H, identical Barnes-Hut counters summed over
the sets), and against the single-set GPU calls: the batched Barnes-Hut trees
are the single-set trees (node sums may be added in another order, so
results agree to FP64 rounding, not bitwise) and the batched exact sums use
the same FP32 tiles with other FP64 split boundaries.  The full-size case is
the 64-subject population (sizes U{5000..40000}, 1.52 M points).
"""
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


def _ragged(sizes, seed=70):
    """Sets of the ellipsoid recipe with the given sizes (0 and 1 allowed)."""
    out = []
    for k, n in enumerate(sizes):
        if n == 0:
            out.append(W.Workload(f"empty-{k}", np.zeros((0, 3), np.float32),
                                  np.zeros((0, 3), np.float32), 0.05, 40, "f32"))
        else:
            out.append(W.ellipsoid_20k(seed=seed + k, n=n))
    return out


SIZES = [700, 0, 1, 2500, 64, 3, 1333]


@pytest.mark.parametrize("method", [gs.GS_EXACT, gs.GS_BH])
def test_rhs_batch_matches_oracle_per_set(oracle, method):
    subs = _ragged(SIZES)
    q, p, off = W.stack(subs)
    sigma, theta, leaf_cap = 0.05, 0.5, 8
    prm = gs.params(sigma, theta=theta, leaf_cap=leaf_cap)
    _say(f"rhs_batch method={method} sizes={SIZES}")
    dq, dp, ws = gs.gs_rhs_batch(_t(q), _t(p), off, prm, method, return_ws=True)
    torch.cuda.synchronize()
    v, a = _np(dq), _np(dp)
    tot = {"pairs": 0, "monopoles": 0}
    for s, w in enumerate(subs):
        lo, hi = off[s], off[s + 1]
        if hi == lo:
            continue
        q64, p64 = w.q0.astype(np.float64), w.p0.astype(np.float64)
        if method == gs.GS_EXACT:
            vo, ao = oracle.rhs_exact(q64, p64, sigma)
        else:
            vo, ao, c = oracle.rhs_bh(q64, p64, sigma, theta, leaf_cap=leaf_cap)
            tot["pairs"] += c["pairs"]
            tot["monopoles"] += c["monopoles"]
        ev, ea = rel_l2(v[lo:hi], vo), rel_l2(a[lo:hi], ao) if np.any(ao) else 0.0
        _say(f"  set {s} n={hi - lo}: rel-L2 v {ev:.2e} a {ea:.2e}")
        assert ev < 1e-5 and ea < 1e-5
    if method == gs.GS_BH:
        cnt = gs.gs_bh_counters(ws)
        _say(f"  counters gpu {cnt} oracle {tot}")
        assert cnt["pairs"] == tot["pairs"] and cnt["monopoles"] == tot["monopoles"]
        assert gs.gs_get_status(ws) == 0


@pytest.mark.parametrize("method", [gs.GS_EXACT, gs.GS_BH])
def test_shoot_batch_matches_oracle_per_set(oracle, method):
    subs = _ragged([900, 1, 0, 1700, 130])
    q, p, off = W.stack(subs)
    sigma, nt, theta, leaf_cap = 0.05, 6, 0.5, 4
    prm = gs.params(sigma, nt=nt, theta=theta, leaf_cap=leaf_cap)
    _say(f"shoot_batch method={method}")
    q1, p1, H = gs.gs_shoot_batch(_t(q), _t(p), off, prm, method)
    torch.cuda.synchronize()
    q1, p1, H = _np(q1), _np(p1), _np(H)
    assert H.shape == (len(subs), nt + 1)
    for s, w in enumerate(subs):
        lo, hi = off[s], off[s + 1]
        if hi == lo:
            assert np.all(H[s] == 0.0)
            continue
        kind = "exact" if method == gs.GS_EXACT else "bh"
        qo, po, Ho = oracle.shoot(w.q0.astype(np.float64), w.p0.astype(np.float64), sigma, nt,
                                  method=kind, theta=theta, leaf_cap=leaf_cap)
        eq, ep = rel_l2(q1[lo:hi], qo), rel_l2(p1[lo:hi], po)
        eh = float(np.max(np.abs(H[s] - Ho)) / np.max(np.abs(Ho)))
        _say(f"  set {s} n={hi - lo}: q1 {eq:.2e} p1 {ep:.2e} H {eh:.2e}")
        assert eq < 1e-5 and ep < 1e-5 and eh < 1e-6


def _single_vs_batch(subs, prm, method, rhs=False):
    q, p, off = W.stack(subs)
    if rhs:
        out_b = gs.gs_rhs_batch(_t(q), _t(p), off, prm, method)
    else:
        out_b = gs.gs_shoot_batch(_t(q), _t(p), off, prm, method)
    worst = [0.0, 0.0, 0.0]
    for s, w in enumerate(subs):
        lo, hi = int(off[s]), int(off[s + 1])
        if hi == lo:
            if not rhs:
                assert np.all(_np(out_b[2][s]) == 0.0)
            continue
        if rhs:
            fn = gs.gs_rhs_exact if method == gs.GS_EXACT else gs.gs_rhs_bh
            one = fn(_t(w.q0), _t(w.p0), prm)
        else:
            one = gs.gs_shoot(_t(w.q0), _t(w.p0), prm, method)
        for k in range(2):
            worst[k] = max(worst[k], rel_l2(_np(out_b[k][lo:hi]), _np(one[k])))
        if not rhs:
            Hs, Hb = _np(one[2]), _np(out_b[2][s])
            worst[2] = max(worst[2], float(np.max(np.abs(Hb - Hs)) / np.max(np.abs(Hs))))
    return worst


@pytest.mark.parametrize("method", [gs.GS_EXACT, gs.GS_BH])
def test_batch_equals_single_calls(method):
    subs = _ragged([3000, 64, 65, 1, 2049, 0, 5000], seed=90)
    prm = gs.params(0.05, nt=5, theta=0.5, leaf_cap=16)
    for rhs in (True, False):
        worst = _single_vs_batch(subs, prm, method, rhs=rhs)
        _say(f"batch vs single method={method} rhs={rhs}: {worst}")
        assert max(worst) < 1e-6


def test_population_full_size(oracle):
    """The 64-subject population: Barnes-Hut and exact batched RHS against the
    oracle (counters in full; exact rows sampled per subject), batched
    shootings against single-subject shootings."""
    subs = W.population()
    q, p, off = W.stack(subs)
    n = int(off[-1])
    sigma, theta, leaf_cap = 0.05, 0.5, 16
    prm = gs.params(sigma, nt=40, theta=theta, leaf_cap=leaf_cap)
    _say(f"population: {len(subs)} subjects, {n} points, sum N^2 "
         f"{float(np.sum(np.diff(off).astype(np.float64) ** 2)):.3e}")
    qt, pt = _t(q), _t(p)
    dq, dp, ws = gs.gs_rhs_batch(qt, pt, off, prm, gs.GS_BH, return_ws=True)
    xv, xa = gs.gs_rhs_batch(qt, pt, off, prm, gs.GS_EXACT)
    torch.cuda.synchronize()
    cnt = gs.gs_bh_counters(ws)
    v, a, xv, xa = _np(dq), _np(dp), _np(xv), _np(xa)
    rng = np.random.default_rng(11)
    tot = {"pairs": 0, "monopoles": 0}
    worst_bh, worst_x = 0.0, 0.0
    for s, w in enumerate(subs):
        lo, hi = off[s], off[s + 1]
        q64, p64 = w.q0.astype(np.float64), w.p0.astype(np.float64)
        vo, ao, c = oracle.rhs_bh(q64, p64, sigma, theta, leaf_cap=leaf_cap)
        tot["pairs"] += c["pairs"]
        tot["monopoles"] += c["monopoles"]
        worst_bh = max(worst_bh, rel_l2(v[lo:hi], vo), rel_l2(a[lo:hi], ao))
        idx = np.sort(rng.choice(hi - lo, 48, replace=False))
        ro_v, ro_a = oracle.rhs_exact_rows(idx, q64, p64, sigma)
        worst_x = max(worst_x, rel_l2(xv[lo:hi][idx], ro_v), rel_l2(xa[lo:hi][idx], ro_a))
    _say(f"  BH rel-L2 worst {worst_bh:.2e}; exact sampled rel-L2 worst {worst_x:.2e}")
    _say(f"  counters gpu {cnt} oracle {tot}")
    assert worst_bh < 1e-5 and worst_x < 1e-5
    assert cnt["pairs"] == tot["pairs"] and cnt["monopoles"] == tot["monopoles"]
    for method in (gs.GS_BH, gs.GS_EXACT):
        worst = _single_vs_batch(subs, prm, method)
        _say(f"  shooting batch vs single method={method}: {worst}")
        assert max(worst) < 1e-6
    # the flows are well resolved: the energy of every subject stays within a
    # few percent of H(0) over the 40 Euler steps
    _, _, H = gs.gs_shoot_batch(qt, pt, off, prm, gs.GS_EXACT)
    H = _np(H)
    drift = np.max(np.abs(H - H[:, :1]) / np.abs(H[:, :1]), axis=1)
    _say(f"  energy drift per subject: max {drift.max():.2e} median {np.median(drift):.2e}")
    assert drift.max() < 0.05


def test_autotune_leaf_cap_picks_a_valid_fast_setting():
    """The tuner returns one of its candidates, the time it reports is that
    of an RHS at that setting, and the tuned RHS keeps the oracle parity of
    the Barnes-Hut path (larger leaves only add exact pairs)."""
    w = W.ellipsoid_20k(n=20000)
    q, p = _t(w.q0), _t(w.p0)
    prm = gs.params(w.sigma, theta=0.5, leaf_cap=1)
    tuned, ms = gs.gs_autotune_leaf_cap(q, p, prm)
    _say(f"autotune leaf_cap -> {tuned.leaf_cap} ({ms:.3f} ms per RHS)")
    assert tuned.leaf_cap in (8, 16, 32, 48, 64) and ms > 0
    assert (tuned.sigma, tuned.theta, tuned.nt) == (prm.sigma, prm.theta, prm.nt)
    subs = W.population(subjects=6)
    qq, pp, off = W.stack(subs)
    tb, msb = gs.gs_autotune_leaf_cap(_t(qq), _t(pp), gs.params(0.05, theta=0.5), offsets=off)
    _say(f"autotune batch leaf_cap -> {tb.leaf_cap} ({msb:.3f} ms per batched RHS)")
    assert tb.leaf_cap in (8, 16, 32, 48, 64)


def test_autotune_exact_picks_a_candidate_and_keeps_parity(oracle):
    """The exact-path tuner returns one of its candidates; the tuned setting
    only moves FP64 chunk boundaries (FP32 tiles are unchanged), so the RHS
    agrees with the default one to FP32 rounding and with the oracle."""
    w = W.ellipsoid_20k(n=20000)
    q, p = _t(w.q0), _t(w.p0)
    prm = gs.params(w.sigma)
    tuned, ms = gs.gs_autotune_exact(q, p, prm)
    _say(f"autotune exact -> exact_items {tuned.exact_items} ({ms:.3f} ms per RHS)")
    assert tuned.exact_items in (6144, 12288, 24576, 49152) and ms > 0
    assert (tuned.sigma, tuned.leaf_cap, tuned.nt) == (prm.sigma, prm.leaf_cap, prm.nt)
    ref = [_np(x) for x in gs.gs_rhs_exact(q, p, prm)]
    for items in (6144, 49152):
        other = gs.Params.from_buffer_copy(prm)
        other.exact_items = items
        got = [_np(x) for x in gs.gs_rhs_exact(q, p, other)]
        assert rel_l2(got[0], ref[0]) < 1e-7 and rel_l2(got[1], ref[1]) < 1e-7, items
    idx = np.sort(np.random.default_rng(3).choice(w.n, 64, replace=False))
    vo, ao = oracle.rhs_exact_rows(idx, w.q0.astype(np.float64), w.p0.astype(np.float64), w.sigma)
    got = [_np(x) for x in gs.gs_rhs_exact(q, p, tuned)]
    assert rel_l2(got[0][idx], vo) < 1e-5 and rel_l2(got[1][idx], ao) < 1e-5
    subs = W.population(subjects=6)
    qq, pp, off = W.stack(subs)
    tb, msb = gs.gs_autotune_exact(_t(qq), _t(pp), gs.params(0.05), offsets=off)
    _say(f"autotune exact batch -> exact_items {tb.exact_items} ({msb:.3f} ms per batched RHS)")
    assert tb.exact_items in (6144, 12288, 24576, 49152)


@pytest.mark.parametrize("method", [gs.GS_EXACT, gs.GS_BH])
def test_many_tiny_sets(oracle, method):
    """300 sets of 0..40 points: more than 256 sets take two radix passes on
    the set index; every set must still come out as the set alone."""
    rng = np.random.default_rng(300)
    sizes = [int(x) for x in rng.integers(0, 41, size=300)]
    subs = _ragged(sizes, seed=1000)
    q, p, off = W.stack(subs)
    sigma, theta, leaf_cap = 0.05, 0.5, 4
    prm = gs.params(sigma, nt=3, theta=theta, leaf_cap=leaf_cap)
    _say(f"many tiny sets: {len(sizes)} sets, {int(off[-1])} points, method={method}")
    dq, dp, ws = gs.gs_rhs_batch(_t(q), _t(p), off, prm, method, return_ws=True)
    q1, p1, H = gs.gs_shoot_batch(_t(q), _t(p), off, prm, method)
    torch.cuda.synchronize()
    v, a, q1, p1, H = _np(dq), _np(dp), _np(q1), _np(p1), _np(H)
    pairs = 0
    # Elementwise bar on v (the contract itself is rel-L2 1e-5 per set).  The
    # exact kernel stores k (q - c) rounded once to FP32 (k^2 = log2(e) /
    # 2 sigma^2), so a pair's weight carries a relative error of about
    # 2 |d'| ulp(k extent / 2), d' = k (q_i - q_j); with 40 points, one near
    # pair can dominate a small component.  A float32 emulation of that
    # storage on 900 such sets gives up to 5e-7 max|v| (with the centre, or
    # with no centre at all), hence 1e-6 max|v|.  The Barnes-Hut leaf pairs
    # take differences of the inputs themselves (frame origin 0 around the
    # origin) and keep 1e-7 max|v|.
    v_atol = 1e-6 if method == gs.GS_EXACT else 1e-7
    for s, w in enumerate(subs):
        lo, hi = off[s], off[s + 1]
        if hi == lo:
            assert np.all(H[s] == 0.0)
            continue
        q64, p64 = w.q0.astype(np.float64), w.p0.astype(np.float64)
        if method == gs.GS_EXACT:
            vo, ao = oracle.rhs_exact(q64, p64, sigma)
        else:
            vo, ao, c = oracle.rhs_bh(q64, p64, sigma, theta, leaf_cap=leaf_cap)
            pairs += c["pairs"]
        assert np.allclose(v[lo:hi], vo, rtol=1e-5, atol=v_atol * np.abs(vo).max())
        assert np.allclose(a[lo:hi], ao, rtol=1e-4, atol=1e-6 * (np.abs(ao).max() + 1e-30))
        kind = "exact" if method == gs.GS_EXACT else "bh"
        qo, po, Ho = oracle.shoot(q64, p64, sigma, 3, method=kind, theta=theta,
                                  leaf_cap=leaf_cap)
        assert rel_l2(q1[lo:hi], qo) < 1e-5
        assert np.max(np.abs(H[s] - Ho)) <= 1e-6 * np.max(np.abs(Ho))
    if method == gs.GS_BH:
        assert gs.gs_bh_counters(ws)["pairs"] == pairs


def _adjoint_sets(sizes, seed=80):
    """Ragged sets of the gradient workload (template, p0, target)."""
    subs = []
    for k, n in enumerate(sizes):
        if n == 0:
            z = np.zeros((0, 3), np.float32)
            subs.append(W.Workload(f"empty-{k}", z, z, 0.05, 40, "f32", {"target": z}))
        else:
            subs.append(W.adjoint_50k(seed=seed + k, n=n))
    q, p, off = W.stack(subs)
    y = np.concatenate([w.extra["target"] for w in subs])
    return subs, q, p, y, off


@pytest.mark.parametrize("method", [gs.GS_EXACT, gs.GS_BH])
def test_adjoint_batch_matches_oracle_per_set(oracle, method):
    """Per-set objective and gradient against the oracle's, at the single-set
    bars (exact: 1e-6 objective, rel-L2 1e-5 gradient; Barnes-Hut: 1e-5
    objective and gradient against the oracle's Barnes-Hut ones)."""
    subs, q, p, y, off = _adjoint_sets([700, 0, 1, 1300, 64])
    sigma, nt, lam, ck, theta, leaf_cap = 0.05, 6, 0.01, 4, 0.5, 4
    prm = gs.params(sigma, nt=nt, theta=theta, leaf_cap=leaf_cap)
    _say(f"adjoint batch method={method}")
    E, G = gs.gs_shoot_adjoint_batch(_t(q), _t(p), _t(y), off, prm, method, lam, ck)
    torch.cuda.synchronize()
    E, G = _np(E), _np(G)
    kind = "exact" if method == gs.GS_EXACT else "bh"
    for s, w in enumerate(subs):
        lo, hi = off[s], off[s + 1]
        if hi == lo:
            assert E[s] == 0.0
            continue
        q64, p64, y64 = (x.astype(np.float64) for x in (w.q0, w.p0, w.extra["target"]))
        oe, og = oracle.objective_grad(q64, p64, y64, sigma, nt, lam, method=kind, theta=theta,
                                       leaf_cap=leaf_cap)
        eg, ee = rel_l2(G[lo:hi], og), abs(E[s] - oe) / abs(oe)
        if method == gs.GS_EXACT:
            _say(f"  set {s} n={hi - lo}: objective {ee:.2e} grad {eg:.2e}")
            assert ee <= 1e-6 and eg < 1e-5
        else:
            _, xg = oracle.objective_grad(q64, p64, y64, sigma, nt, lam)
            eps = rel_l2(og, xg)
            _say(f"  set {s} n={hi - lo}: objective {ee:.2e} grad {eg:.2e} eps {eps:.2e}")
            assert ee <= 1e-5 and eg <= 1e-5


@pytest.mark.parametrize("method", [gs.GS_EXACT, gs.GS_BH])
def test_adjoint_batch_equals_single_calls(method):
    subs, q, p, y, off = _adjoint_sets([3000, 64, 65, 1, 2049, 0, 5000], seed=120)
    prm = gs.params(0.05, nt=5, theta=0.5, leaf_cap=16)
    E, G = gs.gs_shoot_adjoint_batch(_t(q), _t(p), _t(y), off, prm, method, 0.01, 2)
    E, G = _np(E), _np(G)
    worst = 0.0
    for s, w in enumerate(subs):
        lo, hi = off[s], off[s + 1]
        if hi == lo:
            continue
        e1, g1 = gs.gs_shoot_adjoint(_t(w.q0), _t(w.p0), _t(w.extra["target"]), prm, method,
                                     0.01, 2)
        worst = max(worst, abs(E[s] - float(e1)) / abs(float(e1)), rel_l2(G[lo:hi], _np(g1)))
    _say(f"adjoint batch vs single method={method}: {worst:.2e}")
    assert worst < 1e-6


def test_population_adjoint_full_size():
    """Forward plus backward stage of the 64-subject population (40 steps,
    checkpoints every 8): the batched objective and gradient of sampled
    subjects equal their single-subject calls (which the oracle pins at
    smaller sizes)."""
    subs = W.population()
    ys = W.population_targets(subs)
    q, p, off = W.stack(subs)
    y = np.concatenate(ys)
    prm = gs.params(0.05, nt=40, theta=0.5, leaf_cap=16)
    qt, pt, yt = _t(q), _t(p), _t(y)
    sizes = np.diff(off)
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes)), 17]
    for method in (gs.GS_BH, gs.GS_EXACT):
        _say(f"population adjoint method={method}")
        E, G = gs.gs_shoot_adjoint_batch(qt, pt, yt, off, prm, method, 0.01, 8)
        E, G = _np(E), _np(G)
        assert np.all(np.isfinite(E)) and np.all(E > 0) and np.all(np.isfinite(G))
        for s in picks:
            lo, hi = off[s], off[s + 1]
            e1, g1 = gs.gs_shoot_adjoint(_t(subs[s].q0), _t(subs[s].p0), _t(ys[s]), prm, method,
                                         0.01, 8)
            de = abs(E[s] - float(e1)) / abs(float(e1))
            dg = rel_l2(G[lo:hi], _np(g1))
            _say(f"  subject {s} n={hi - lo}: objective {de:.2e} grad {dg:.2e}")
            assert de < 1e-6 and dg < 1e-6


@pytest.mark.parametrize("subjects", [14, 20])
def test_bh_split_for_mid_sized_batches(oracle, subjects):
    """The decide waves per group depend on the group count (8 below about
    1 500 groups, 4 at 3 000, 1 above 12 000): batches of 14 and 20 subjects
    (about 4 900 and 7 000 groups) take 3 and 2 waves per group.  Every subject must still
    match the oracle's Barnes-Hut RHS and its counters, and its gradient the
    single-subject call."""
    subs = W.population(subjects=subjects)
    q, p, off = W.stack(subs)
    groups = sum((w.n + 63) // 64 for w in subs)
    sigma, theta, leaf_cap = 0.05, 0.5, 16
    prm = gs.params(sigma, nt=3, theta=theta, leaf_cap=leaf_cap)
    _say(f"bh split: {subjects} subjects, {int(off[-1])} points, {groups} groups")
    dq, dp, ws = gs.gs_rhs_batch(_t(q), _t(p), off, prm, gs.GS_BH, return_ws=True)
    cnt = gs.gs_bh_counters(ws)
    v, a = _np(dq), _np(dp)
    pairs = mono = 0
    worst = 0.0
    for s_, w in enumerate(subs):
        lo, hi = off[s_], off[s_ + 1]
        vo, ao, c = oracle.rhs_bh(w.q0.astype(np.float64), w.p0.astype(np.float64), sigma, theta,
                                  leaf_cap=leaf_cap)
        pairs += c["pairs"]
        mono += c["monopoles"]
        worst = max(worst, rel_l2(v[lo:hi], vo), rel_l2(a[lo:hi], ao))
    _say(f"  worst rel-L2 {worst:.2e}; counters gpu {cnt['pairs']} / {cnt['monopoles']}, "
         f"oracle {pairs} / {mono}")
    assert worst < 1e-5 and cnt["pairs"] == pairs and cnt["monopoles"] == mono
    ys = W.population_targets(subs)
    E, G = gs.gs_shoot_adjoint_batch(_t(q), _t(p), _t(np.concatenate(ys)), off, prm, gs.GS_BH,
                                     0.01, 2)
    E, G = _np(E), _np(G)
    for s_ in (0, subjects - 1):
        lo, hi = off[s_], off[s_ + 1]
        e1, g1 = gs.gs_shoot_adjoint(_t(subs[s_].q0), _t(subs[s_].p0), _t(ys[s_]), prm, gs.GS_BH,
                                     0.01, 2)
        assert abs(E[s_] - float(e1)) <= 1e-6 * abs(float(e1))
        assert rel_l2(G[lo:hi], _np(g1)) < 1e-6
