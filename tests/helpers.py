"""Independent small-size formulations used to pin the oracle.

These are written from the definitions, not from the oracle's code: the
Hamiltonian through an explicit 3N x 3N kernel matrix, its derivatives through
torch's float64 autograd, and the Euler loop as plain torch code.  They are
only usable at small N.
"""
from __future__ import annotations

import numpy as np
import torch


def kernel_matrix(q, sigma):
    """K(q) of Sec. 2.1: N x N blocks G(|q_i - q_j|) I_3 (as a 3N x 3N array)."""
    q = np.asarray(q, dtype=np.float64)
    d2 = ((q[:, None, :] - q[None, :, :]) ** 2).sum(-1)
    g = np.exp(-d2 / (2.0 * sigma * sigma))
    return np.kron(g, np.eye(3))


def half_energy_torch(q, p, sigma):
    d = q[:, None, :] - q[None, :, :]
    g = torch.exp(-(d * d).sum(-1) / (2.0 * sigma * sigma))
    return 0.5 * torch.einsum("ij,ic,jc->", g, p, p)


def rhs_autograd(q, p, sigma):
    """(dH/dp, -dH/dq) of H = 1/2 <p, K(q) p> by float64 autograd."""
    qt = torch.tensor(np.asarray(q, np.float64), requires_grad=True)
    pt = torch.tensor(np.asarray(p, np.float64), requires_grad=True)
    h = half_energy_torch(qt, pt, sigma)
    gq, gp = torch.autograd.grad(h, (qt, pt))
    return gp.numpy(), (-gq).numpy()


def euler_objective_torch(q0, p0, y, sigma, nt, lam):
    """Objective |q(1) - y|^2 / n + lam <p0, K(q0) p0> through the Euler loop,
    with the RHS from autograd of the Hamiltonian; returns (E, dE/dp0)."""
    q = torch.tensor(np.asarray(q0, np.float64))
    p0t = torch.tensor(np.asarray(p0, np.float64), requires_grad=True)
    yt = torch.tensor(np.asarray(y, np.float64))
    n = q.shape[0]
    dt = 1.0 / nt
    p = p0t
    for _ in range(nt):
        qv = q if q.requires_grad else q.clone().requires_grad_(True)
        h = half_energy_torch(qv, p, sigma)
        gq, gp = torch.autograd.grad(h, (qv, p), create_graph=True)
        q, p = qv + dt * gp, p - dt * gq
    e = ((q - yt) ** 2).sum() / n + lam * 2.0 * half_energy_torch(
        torch.tensor(np.asarray(q0, np.float64)), p0t, sigma)
    (g,) = torch.autograd.grad(e, (p0t,))
    return float(e), g.numpy()


def rhs_numpy(q, p, sigma):
    """Exact RHS from the explicit kernel matrix (v = K p) and the
    closed-form q-gradient; independent of the oracle's loop order."""
    q = np.asarray(q, np.float64)
    p = np.asarray(p, np.float64)
    d = q[:, None, :] - q[None, :, :]
    g = np.exp(-(d * d).sum(-1) / (2 * sigma * sigma))
    v = g @ p
    s = p @ p.T
    a = ((g * s)[:, :, None] * d).sum(1) / (sigma * sigma)
    return v, a


def rel_l2(x, y):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    den = np.linalg.norm(y)
    return float(np.linalg.norm(x - y) / (den if den > 0 else 1.0))


def morton_interleave(cx, cy, cz, bits):
    """Interleave `bits` low bits of each axis (x highest) into one integer."""
    out = 0
    for b in range(bits - 1, -1, -1):
        out = (out << 3) | (((cx >> b) & 1) << 2) | (((cy >> b) & 1) << 1) | ((cz >> b) & 1)
    return out


def canonical_octree(ic, leaf_cap, levels=21):
    """Brute-force node set of the octree defined on integer coordinates:
    a node is a non-empty cell whose parent holds more than leaf_cap points
    (and lies above the deepest level).  Returns {(level, morton_prefix):
    sorted member tuple}."""
    ic = np.asarray(ic, dtype=np.int64)
    nodes = {}
    stack = [(0, 0, 0, 0, tuple(range(ic.shape[0])))]
    while stack:
        lv, px, py, pz, members = stack.pop()
        nodes[(lv, morton_interleave(px, py, pz, lv))] = members
        if len(members) <= leaf_cap or lv == levels:
            continue
        groups = {}
        sh = levels - lv - 1
        for m in members:
            key = ((ic[m, 0] >> sh) & 1, (ic[m, 1] >> sh) & 1, (ic[m, 2] >> sh) & 1)
            groups.setdefault(key, []).append(m)
        for (bx, by, bz), mem in groups.items():
            stack.append((lv + 1, 2 * px + bx, 2 * py + by, 2 * pz + bz, tuple(sorted(mem))))
    return nodes
