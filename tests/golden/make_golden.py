"""Write stored oracle results for workloads too large to recompute in a test
(or in the benchmark, which never runs the oracle outside its CPU-baseline
leg).

    python tests/golden/make_golden.py ellipsoids8_200k_exact [more jobs]

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


def _rows(rng_seed, n, k):
    return np.sort(np.random.default_rng(rng_seed).choice(n, min(k, n), replace=False))


def ellipsoid_20k_rhs():
    """One right-hand side of ellipsoid-20k: exact, and Barnes-Hut at each
    opening angle of that workload with leaf_cap 1 and 48 (sampled rows)."""
    w = W.ellipsoid_20k()
    q, p = w.q0.astype(np.float64), w.p0.astype(np.float64)
    t0 = time.time()
    idx = _rows(2020, w.n, 2048)
    v, a = O.rhs_exact_rows(idx, q, p, w.sigma)
    out = dict(idx=idx, v_exact=v, a_exact=a, sigma=w.sigma, digest=input_digest(w.q0, w.p0))
    for th in (0.3, 0.5, 0.8):
        for lc in (1, 48):
            vb, ab, _ = O.rhs_bh(q, p, w.sigma, th, leaf_cap=lc)
            out[f"v_bh_{th}_{lc}"] = vb[idx]
            out[f"a_bh_{th}_{lc}"] = ab[idx]
    out["oracle_seconds"] = time.time() - t0
    return out


def ellipsoids8_200k_field():
    """Velocity field of the 200k ellipsoids at 200k uniform points (sampled
    target rows)."""
    w = W.ellipsoids_200k()
    x = W.field_targets()
    idx = _rows(2021, x.shape[0], 2048)
    t0 = time.time()
    v = O.field_exact(x[idx].astype(np.float64), w.q0.astype(np.float64),
                      w.p0.astype(np.float64), w.sigma)
    return dict(idx=idx, v=v, sigma=w.sigma, digest=input_digest(w.q0, w.p0, x),
                oracle_seconds=time.time() - t0)


def adjoint_50k(theta=0.5, leaf_cap=64):
    """Objective and gradient of the 50k gradient workload, exact and
    Barnes-Hut (sampled gradient rows)."""
    w = W.adjoint_50k()
    q, p = w.q0.astype(np.float64), w.p0.astype(np.float64)
    y = w.extra["target"].astype(np.float64)
    idx = _rows(2022, w.n, 4096)
    t0 = time.time()
    out = dict(idx=idx, theta=theta, leaf_cap=leaf_cap, lam=w.extra["lam"], nt=w.nt,
               digest=input_digest(w.q0, w.p0, w.extra["target"]))
    for method in ("exact", "bh"):
        e, g = O.objective_grad(q, p, y, w.sigma, w.nt, w.extra["lam"], method=method,
                                theta=theta, leaf_cap=leaf_cap)
        out[f"E_{method}"] = e
        out[f"g_{method}"] = g[idx]
    out["oracle_seconds"] = time.time() - t0
    return out


POP_SUBJECTS = (0, 21, 42, 63)


def population_subjects(theta=0.5, leaf_cap=64):
    """Shooting (exact and Barnes-Hut) and objective / gradient of four
    subjects of the 64-subject population (sampled rows, full H)."""
    subs = W.population()
    ys = W.population_targets(subs)
    out = dict(subjects=np.array(POP_SUBJECTS), theta=theta, leaf_cap=leaf_cap)
    t0 = time.time()
    dig = []
    for s in POP_SUBJECTS:
        w = subs[s]
        q, p, y = (a.astype(np.float64) for a in (w.q0, w.p0, ys[s]))
        idx = _rows(3000 + s, w.n, 1024)
        out[f"idx_{s}"] = idx
        for method in ("exact", "bh"):
            q1, p1, H = O.shoot(q, p, w.sigma, w.nt, method=method, theta=theta,
                                leaf_cap=leaf_cap)
            out[f"q1_{method}_{s}"], out[f"p1_{method}_{s}"] = q1[idx], p1[idx]
            out[f"H_{method}_{s}"] = H
            e, g = O.objective_grad(q, p, y, w.sigma, w.nt, 0.01, method=method, theta=theta,
                                    leaf_cap=leaf_cap)
            out[f"E_{method}_{s}"] = e
            out[f"g_{method}_{s}"] = g[idx]
        dig.append(input_digest(w.q0, w.p0, ys[s]))
        print("  subject", s, w.n, f"{time.time() - t0:.0f}s", flush=True)
    out["digest"] = input_digest(*[np.frombuffer(d.encode(), np.uint8) for d in dig])
    out["oracle_seconds"] = time.time() - t0
    return out


JOBS = {
    "ellipsoid_20k_rhs": ellipsoid_20k_rhs,
    "ellipsoids8_200k_field": ellipsoids8_200k_field,
    "adjoint_50k_grad": adjoint_50k,
    "population_subjects": population_subjects,
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
