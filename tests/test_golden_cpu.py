"""Stored oracle results (tests/golden/*.npz) still describe today's inputs:
the input digest matches the seeded generator, the sample indices are valid,
and the stored energies behave as the Euler scheme must (finite, positive,
drift of a few percent over 40 steps at this resolution)."""
import glob
import hashlib
import os

import numpy as np
import pytest

from paper_1907_04834_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FILES = sorted(glob.glob(os.path.join(GOLD, "ellipsoids8_200k_exact.npz")) +
               glob.glob(os.path.join(GOLD, "ellipsoids8_200k_bh05_*.npz")))


def _digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


@pytest.fixture(scope="module")
def digest():
    w = W.ellipsoids_200k()
    return _digest(w.q0, w.p0), w.n


@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f) for f in FILES])
def test_golden_file_matches_generator(path, digest):
    g = np.load(path)  # allow_pickle stays False: plain arrays only
    dig, n = digest
    assert str(g["digest"]) == dig
    idx = g["idx"]
    assert idx.shape == (4096,) and np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < n
    H = g["H"]
    assert H.shape == (int(g["nt"]) + 1,) and np.all(np.isfinite(H)) and np.all(H > 0)
    assert abs(H[-1] - H[0]) / H[0] < 0.1
    assert np.all(np.isfinite(g["q1"])) and np.all(np.isfinite(g["p1"]))


def test_golden_bh_close_to_exact():
    """The stored Barnes-Hut shootings differ from the stored exact one by a
    small amount (the approximation error at theta 0.5), and not by zero."""
    ex = os.path.join(GOLD, "ellipsoids8_200k_exact.npz")
    bhs = [f for f in FILES if "_bh05_" in f]
    if not os.path.exists(ex) or not bhs:
        pytest.skip("golden files not generated")
    gx = np.load(ex)
    for f in bhs:
        gb = np.load(f)
        e = np.linalg.norm(gb["p1"] - gx["p1"]) / np.linalg.norm(gx["p1"])
        assert 1e-6 < e < 0.1, (f, e)


def _load(name):
    path = os.path.join(GOLD, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"{name}.npz not written (tests/golden/make_golden.py {name})")
    return np.load(path)


def test_golden_rhs_20k_matches_generator():
    g = _load("ellipsoid_20k_rhs")
    w = W.ellipsoid_20k()
    assert str(g["digest"]) == _digest(w.q0, w.p0)
    idx = g["idx"]
    assert np.all(np.diff(idx) > 0) and idx[-1] < w.n
    for th in (0.3, 0.5, 0.8):
        for lc in (1, 48):
            v, a = g[f"v_bh_{th}_{lc}"], g[f"a_bh_{th}_{lc}"]
            assert v.shape == (len(idx), 3) and np.all(np.isfinite(v)) and np.all(np.isfinite(a))
            # the approximation moves the result by a small fraction only
            assert np.linalg.norm(v - g["v_exact"]) < 0.05 * np.linalg.norm(g["v_exact"])


def test_golden_field_matches_generator():
    g = _load("ellipsoids8_200k_field")
    w = W.ellipsoids_200k()
    x = W.field_targets()
    assert str(g["digest"]) == _digest(w.q0, w.p0, x)
    assert g["v"].shape == (len(g["idx"]), 3) and np.all(np.isfinite(g["v"]))


def test_golden_adjoint_matches_generator():
    g = _load("adjoint_50k_grad")
    w = W.adjoint_50k()
    assert str(g["digest"]) == _digest(w.q0, w.p0, w.extra["target"])
    for m in ("exact", "bh"):
        assert np.isfinite(float(g[f"E_{m}"])) and float(g[f"E_{m}"]) > 0
        assert np.all(np.isfinite(g[f"g_{m}"]))
    # Barnes-Hut objective within a few percent of the exact one
    assert abs(float(g["E_bh"]) - float(g["E_exact"])) < 0.05 * float(g["E_exact"])


def test_golden_population_subjects_match_generator():
    g = _load("population_subjects")
    subs = W.population()
    ys = W.population_targets(subs)
    dig = [_digest(subs[s].q0, subs[s].p0, ys[s]) for s in g["subjects"]]
    assert str(g["digest"]) == _digest(*[np.frombuffer(d.encode(), np.uint8) for d in dig])
    for s in g["subjects"]:
        for m in ("exact", "bh"):
            H = g[f"H_{m}_{s}"]
            assert np.all(np.isfinite(H)) and abs(H[-1] - H[0]) < 0.1 * H[0]
