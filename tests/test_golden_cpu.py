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
FILES = sorted(glob.glob(os.path.join(GOLD, "ellipsoids8_200k_*.npz")))


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
