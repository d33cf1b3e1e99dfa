"""Full-size shooting (200k points on 8 ellipsoids, 40 steps) against stored
FP64 oracle results.

The oracle's exact shooting at this size takes over an hour on a CPU, so its
results are stored (tests/golden/*.npz, written by make_golden.py from the
oracle alone): a fixed sample of 4096 rows of q(1) and p(1) and the whole
energy history H[0..40].  The GPU runs the same launch configuration as the
benchmark.  Bars: exact FP32 path rel-L2 1e-5 on q(1) and p(1), 1e-6 on H;
Barnes-Hut path max(1e-5, 0.1 eps_theta) against the oracle's Barnes-Hut
shooting, eps_theta being the oracle's own Barnes-Hut vs exact difference.
"""
import hashlib
import os

import numpy as np
import pytest
import torch

from helpers import rel_l2
from paper_1907_04834_amd import gs
from paper_1907_04834_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _load(name):
    path = os.path.join(GOLD, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"{name}.npz not generated")
    return np.load(path)


@pytest.fixture(scope="module")
def work():
    w = W.ellipsoids_200k()
    return w, _digest(w.q0, w.p0)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def test_exact_shooting_200k_matches_stored_oracle(work):
    w, dig = work
    g = _load("ellipsoids8_200k_exact")
    assert str(g["digest"]) == dig
    print("shoot exact n=200000 vs stored oracle", flush=True)
    prm = gs.params(w.sigma, nt=w.nt)
    q1, p1, H = gs.gs_shoot(torch.from_numpy(w.q0).to(DEV), torch.from_numpy(w.p0).to(DEV), prm,
                            gs.GS_EXACT)
    idx = g["idx"]
    eq, ep = rel_l2(_np(q1)[idx], g["q1"]), rel_l2(_np(p1)[idx], g["p1"])
    eh = float(np.max(np.abs(_np(H) - g["H"])) / np.max(np.abs(g["H"])))
    print(f"  q1 {eq:.2e} p1 {ep:.2e} H {eh:.2e}", flush=True)
    assert eq < 1e-5 and ep < 1e-5 and eh < 1e-6


@pytest.mark.parametrize("leaf_cap", [1, 64])
def test_bh_shooting_200k_matches_stored_oracle(work, leaf_cap):
    w, dig = work
    gx = _load("ellipsoids8_200k_exact")
    gb = _load(f"ellipsoids8_200k_bh05_lc{leaf_cap}")
    assert str(gb["digest"]) == dig and np.array_equal(gb["idx"], gx["idx"])
    eps_q, eps_p = rel_l2(gb["q1"], gx["q1"]), rel_l2(gb["p1"], gx["p1"])
    print(f"shoot bh n=200000 leaf_cap={leaf_cap}: eps_theta q {eps_q:.2e} p {eps_p:.2e}",
          flush=True)
    prm = gs.params(w.sigma, nt=w.nt, theta=0.5, leaf_cap=leaf_cap)
    q1, p1, H = gs.gs_shoot(torch.from_numpy(w.q0).to(DEV), torch.from_numpy(w.p0).to(DEV), prm,
                            gs.GS_BH)
    idx = gb["idx"]
    eq, ep = rel_l2(_np(q1)[idx], gb["q1"]), rel_l2(_np(p1)[idx], gb["p1"])
    eh = float(np.max(np.abs(_np(H) - gb["H"])) / np.max(np.abs(gb["H"])))
    print(f"  vs oracle BH: q1 {eq:.2e} p1 {ep:.2e} H {eh:.2e}", flush=True)
    assert eq < max(1e-5, 0.1 * eps_q) and ep < max(1e-5, 0.1 * eps_p)
    assert eh < 1e-5
