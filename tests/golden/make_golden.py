"""Write stored oracle results for workloads too large to recompute in a test.

    python tests/golden/make_golden.py ellipsoids8_200k_exact

Calls only the FP64 oracle (oracle/oracle.py) on inputs from the seeded
workload generators, and stores a fixed random sample of output rows (the
sample indices are stored with them) plus the full energy history H[0..nt]
as a numpy .npz (no pickles).
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1907_04834_amd import workloads as W  # noqa: E402

SAMPLE = 4096


def input_digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def ellipsoids8_200k(method: str, theta: float = 0.5, leaf_cap: int = 1):
    w = W.ellipsoids_200k()
    q, p = w.q0.astype(np.float64), w.p0.astype(np.float64)
    t0 = time.time()
    q1, p1, H = O.shoot(q, p, w.sigma, w.nt, method=method, theta=theta, leaf_cap=leaf_cap)
    secs = time.time() - t0
    idx = np.sort(np.random.default_rng(12345).choice(w.n, SAMPLE, replace=False))
    return dict(idx=idx, q1=q1[idx], p1=p1[idx], H=H, sigma=w.sigma, nt=w.nt,
                theta=theta, leaf_cap=leaf_cap, digest=input_digest(w.q0, w.p0),
                oracle_seconds=secs, threads=int(os.environ.get("OMP_NUM_THREADS", "0")))


JOBS = {
    "ellipsoids8_200k_exact": lambda: ellipsoids8_200k("exact"),
    "ellipsoids8_200k_bh05_lc1": lambda: ellipsoids8_200k("bh", 0.5, 1),
    "ellipsoids8_200k_bh05_lc64": lambda: ellipsoids8_200k("bh", 0.5, 64),
}


if __name__ == "__main__":
    for name in sys.argv[1:]:
        res = JOBS[name]()
        out = os.path.join(HERE, name + ".npz")
        np.savez(out, **{k: np.asarray(v) for k, v in res.items()})
        print(name, "->", out, f"{res['oracle_seconds']:.1f}s", flush=True)
