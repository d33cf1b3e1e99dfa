"""Seeded synthetic inputs for point-set geodesic shooting.

The paper evaluates on surface point sets: Poisson-disk samples of a medial
temporal lobe cortex mesh (Sec. 3.2) and small synthetic curves and meshes
(Sec. 3.1).  Neither data set is available, so these generators stand in for
them with point sets of the same kind: points spread over closed surfaces
(spheres, ellipsoids, unions of ellipsoids) with small normal jitter, and
initial momenta that are either i.i.d. Gaussian or a smooth field.

This module holds no part of the method's arithmetic: it only draws points,
momenta, targets and directions.  Both the GPU library's tests and the oracle's
tests take their inputs from here.  Every draw uses numpy's PCG64
(``numpy.random.default_rng(seed)``) in a fixed order, in float64; FP32
workloads are rounded to float32 once, and the oracle receives exactly those
float32 values promoted to float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _unit_sphere(rng, n):
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def sphere_points(rng, n, jitter=0.01):
    """Points on the unit sphere plus isotropic N(0, jitter^2) noise."""
    u = _unit_sphere(rng, n)
    return u + jitter * rng.standard_normal((n, 3))


def ellipsoid_surface(rng, n, axes, normal_jitter=0.0):
    """n points uniform by area on the ellipsoid with the given semi-axes,
    optionally moved along the unit normal by N(0, normal_jitter^2).

    Area-uniform by rejection: u uniform on S^2 maps to x = axes * u; the area
    element of that map is proportional to |axes^-1 * u|, so u is accepted with
    probability min(axes) * |u / axes| <= 1."""
    axes = np.asarray(axes, dtype=np.float64)
    out = np.empty((0, 3))
    amin = axes.min()
    while out.shape[0] < n:
        m = max(2 * (n - out.shape[0]), 1024)
        u = _unit_sphere(rng, m)
        w = amin * np.linalg.norm(u / axes, axis=1)
        keep = rng.random(m) < w
        out = np.concatenate([out, u[keep] * axes])
    x = out[:n]
    if normal_jitter > 0.0:
        nrm = x / axes**2
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        x = x + nrm * (normal_jitter * rng.standard_normal((n, 1)))
    return x


def ellipsoid_area(axes):
    """Surface area of an ellipsoid (Knud Thomsen's approximation, rel. err
    about 1%); used only to split a point budget between shapes."""
    a, b, c = (float(x) for x in axes)
    pw = 1.6075
    return 4.0 * np.pi * (((a * b) ** pw + (a * c) ** pw + (b * c) ** pw) / 3.0) ** (1.0 / pw)


def random_rotation(rng):
    """Uniform random rotation (QR of a Gaussian matrix with sign fix)."""
    z = rng.standard_normal((3, 3))
    qm, r = np.linalg.qr(z)
    qm = qm * np.sign(np.diag(r))
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def ellipsoid_union(rng, n, k=8, rmin=0.1, rmax=0.4):
    """n points on the union of k randomly placed, randomly rotated ellipsoids
    inside [0, 1]^3 (semi-axes U[rmin, rmax]; centre U[rho, 1 - rho]^3 with rho
    the largest semi-axis; points split between shapes by area)."""
    axes = rng.uniform(rmin, rmax, size=(k, 3))
    rots = [random_rotation(rng) for _ in range(k)]
    centres = np.stack([rng.uniform(a.max(), 1.0 - a.max(), size=3) for a in axes])
    area = np.array([ellipsoid_area(a) for a in axes])
    counts = rng.multinomial(n, area / area.sum())
    parts = []
    for i in range(k):
        x = ellipsoid_surface(rng, int(counts[i]), axes[i])
        parts.append(x @ rots[i].T + centres[i])
    return np.concatenate(parts)


def bump_field(rng, x, m=16, width=0.15, amp=5e-4):
    """Smooth vector field sum_m A_m exp(-|x - c_m|^2 / (2 width^2)),
    c_m ~ U[0,1]^3, A_m ~ N(0, amp^2 I_3), sampled at x."""
    c = rng.random((m, 3))
    A = amp * rng.standard_normal((m, 3))
    d2 = ((x[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    return np.exp(-d2 / (2.0 * width * width)) @ A


@dataclass
class Workload:
    name: str
    q0: np.ndarray
    p0: np.ndarray
    sigma: float
    nt: int
    dtype: str
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.q0.shape[0])


def _round(x, dtype):
    if dtype == "f32":
        return np.ascontiguousarray(x.astype(np.float32))
    return np.ascontiguousarray(x.astype(np.float64))


def sphere_1024(seed=1, n=1024):
    """Exact shooting in FP64: unit sphere + N(0,0.01^2) jitter, p0 ~ N(0,
    0.05^2), sigma 0.2, 20 Euler steps."""
    rng = np.random.default_rng(seed)
    q = sphere_points(rng, n)
    p = 0.05 * rng.standard_normal((n, 3))
    return Workload("sphere-1024-fp64", _round(q, "f64"), _round(p, "f64"),
                    0.2, 20, "f64")


def ellipsoid_20k(seed=2, n=20000):
    """Noisy ellipsoid (1.0, 0.6, 0.4), area-uniform, N(0,0.005^2) normal
    jitter, p0 ~ N(0, 0.02^2), sigma 0.05, 40 steps, FP32."""
    rng = np.random.default_rng(seed)
    q = ellipsoid_surface(rng, n, (1.0, 0.6, 0.4), 0.005)
    p = 0.02 * rng.standard_normal((n, 3))
    return Workload("ellipsoid-20k", _round(q, "f32"), _round(p, "f32"), 0.05, 40,
                    "f32", {"thetas": (0.3, 0.5, 0.8)})


def ellipsoids_200k(seed=3, n=200000):
    """Union of 8 ellipsoids (semi-axes U[0.1,0.4]) in [0,1]^3, p0 a smooth
    field of 16 Gaussian bumps (width 0.15), sigma 0.02, 40 steps, FP32."""
    rng = np.random.default_rng(seed)
    q = ellipsoid_union(rng, n)
    p = bump_field(rng, q)
    return Workload("ellipsoids8-200k", _round(q, "f32"), _round(p, "f32"), 0.02,
                    40, "f32", {"theta": 0.5})


def adjoint_50k(seed=4, n=50000):
    """Gradient workload: template on the noisy ellipsoid, momenta
    p0 ~ N(0, 0.01^2), target = template moved by a smooth displacement (16
    Gaussian bumps of width 0.3, amplitude 0.03), sigma 0.05, 40 steps,
    lambda 0.01, checkpoints every 8 steps."""
    rng = np.random.default_rng(seed)
    q = ellipsoid_surface(rng, n, (1.0, 0.6, 0.4), 0.005)
    p = 0.01 * rng.standard_normal((n, 3))
    y = q + bump_field(rng, q, m=16, width=0.3, amp=0.03)
    return Workload("adjoint-50k", _round(q, "f32"), _round(p, "f32"), 0.05, 40,
                    "f32", {"target": _round(y, "f32"), "lam": 0.01, "ckpt": 8})


def population(seed=5000, subjects=64, nmin=5000, nmax=40000):
    """Batched population: subjects with n ~ U{nmin..nmax}, each a noisy
    ellipsoid (semi-axes 1, 0.6, 0.4, normal jitter 0.005) with its own
    smooth p0: 16 Gaussian bumps of width 0.3 (0.15 after mapping the
    ellipsoid's box to [0,1]^3) and amplitude 20 / n, so that the mean speed
    |v| is about sigma at every size; sigma 0.05, 40 steps.  (Independent
    N(0, 0.02^2) momenta let the forward-Euler flow of some dense subjects
    blow up within 40 steps.)"""
    out = []
    sizes = np.random.default_rng(seed).integers(nmin, nmax + 1, size=subjects)
    for s in range(subjects):
        rng = np.random.default_rng(seed + 1 + s)
        n = int(sizes[s])
        q = ellipsoid_surface(rng, n, (1.0, 0.6, 0.4), 0.005)
        p = bump_field(rng, (q + 1.0) / 2.0, m=16, width=0.15, amp=20.0 / n)
        out.append(Workload(f"subject-{s}", _round(q, "f32"), _round(p, "f32"),
                            0.05, 40, "f32"))
    return out


def population_targets(subjects, seed=6000):
    """Registration targets of a population: each subject's template moved
    by its own smooth displacement (16 Gaussian bumps of width 0.3,
    amplitude 0.03), as the target of the gradient workload."""
    out = []
    for s, w in enumerate(subjects):
        rng = np.random.default_rng(seed + s)
        q = w.q0.astype(np.float64)
        y = q + bump_field(rng, q, m=16, width=0.3, amp=0.03) if w.n else q
        out.append(_round(y, "f32"))
    return out


def stack(subjects):
    """Concatenates the point sets of a batch: (q, p, offsets) with set s in
    rows offsets[s]..offsets[s+1] (float32 (N, 3) arrays, int64 offsets)."""
    sizes = [w.n for w in subjects]
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    q = np.concatenate([w.q0 for w in subjects]) if subjects else np.zeros((0, 3), np.float32)
    p = np.concatenate([w.p0 for w in subjects]) if subjects else np.zeros((0, 3), np.float32)
    return np.ascontiguousarray(q), np.ascontiguousarray(p), offsets


def field_targets(n=200000, seed=7):
    """Points at which the velocity field is evaluated: uniform in [0, 1]^3
    (the box of the 200k ellipsoids), FP32."""
    rng = np.random.default_rng(seed)
    return _round(rng.random((n, 3)), "f32")


def directions(seed, n, k):
    """k unit directions in R^(3n) (for finite-difference checks)."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((k, n, 3))
    return u / np.linalg.norm(u.reshape(k, -1), axis=1)[:, None, None]


def scaled(w: Workload, n: int, seed: int | None = None) -> Workload:
    """A smaller draw of the same workload family (same recipe, n points)."""
    gen = {"sphere-1024-fp64": sphere_1024, "ellipsoid-20k": ellipsoid_20k,
           "ellipsoids8-200k": ellipsoids_200k, "adjoint-50k": adjoint_50k}[w.name]
    return gen(n=n) if seed is None else gen(seed=seed, n=n)
