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


# ---------------------------------------------------------------------------
# Independent Barnes-Hut evaluation (forward and backward stage), written from
# the definition: the node set is the brute-force set of non-empty Morton cells
# above (canonical_octree), each node's statistics are plain numpy reductions
# over its members, and every target applies the decision rule (Sec. 2.2:
# far from the node's tight box by at least kappa*sigma; opening angle
# s_k < theta |x - C_k|; a node of one point is never approximated).  Nodes
# are visited breadth-first with all the targets that reach them at once, so
# the evaluation order differs from the oracle's depth-first walk.
# ---------------------------------------------------------------------------
LEVELS = 21


def int_coords_np(q):
    """21-bit integer coordinates, c = min(2^21 - 1, floor((q - lo) 2^21 / E))
    in FP64 (zero when the extent E is zero)."""
    q = np.asarray(q, np.float64)
    lo = q.min(0)
    e = float((q.max(0) - lo).max())
    if e == 0.0:
        return np.zeros(q.shape, np.int64)
    s = 2.0 ** LEVELS / e
    f = np.floor((q - lo) * s)
    return np.minimum(f, 2.0 ** LEVELS - 1).astype(np.int64)


def _tree(q, leaf_cap):
    """{(level, prefix): member index array}, children lists, leaf flags."""
    n = q.shape[0]
    ic = int_coords_np(q)
    if n == 0:
        return {}, {}, {}
    if (ic == 0).all() and float((q.max(0) - q.min(0)).max()) == 0.0:
        nodes = {(0, 0): tuple(range(n))}  # zero extent: the root is one leaf
        return nodes, {(0, 0): []}, {(0, 0): True}
    nodes = canonical_octree(ic, leaf_cap, LEVELS)
    kids = {k: [] for k in nodes}
    for (lv, pf) in nodes:
        if lv > 0:
            kids[(lv - 1, pf >> 3)].append((lv, pf))
    leaf = {k: len(kids[k]) == 0 for k in nodes}
    for k in kids:
        kids[k].sort()
    return nodes, kids, leaf


def deepest_set(seed=11):
    """Eight points at the corners of a cube of half-side 2^-k around one
    centre for every k = 2..22 (all FP32-exact), plus two corners fixing the
    box to [0, 1]^3: with leaf_cap 1 the octree reaches level 21, the
    deepest the 21-bit coordinates allow.  Returns FP32 (q, p)."""
    c = np.array([0.40625, 0.59375, 0.53125])
    pts = [np.zeros(3), np.ones(3)]
    for k in range(2, 23):
        for cx in (-1.0, 1.0):
            for cy in (-1.0, 1.0):
                for cz in (-1.0, 1.0):
                    pts.append(c + 2.0 ** -k * np.array([cx, cy, cz]))
    q = np.array(pts, np.float32)
    p = (0.1 * np.random.default_rng(seed).standard_normal(q.shape)).astype(np.float32)
    return q, p


def _adjoint_pairs(xq, xp, xa, xb, qj, pj, aj, bj, wj, sigma):
    """Backward-stage pair terms of targets (rows of xq..xb) against sources
    (rows of qj..bj, each standing for wj[j] identical points), summed over
    the sources:  with d = x - q_j, G = exp(-|d|^2 / 2 sigma^2), s = p_x . p_j,
    db = beta_x - beta_j,
      g_q = sigma^-2 sum_j w_j G { -d [p_j . alpha_x + p_x . alpha_j]
                                    + s [db - d (d . db) / sigma^2] }
      g_p = sum_j w_j G alpha_j + sigma^-2 sum_j w_j G p_j (d . db)."""
    s2 = sigma * sigma
    d = xq[:, None, :] - qj[None, :, :]
    g = np.exp(-(d * d).sum(-1) / (2.0 * s2)) * wj[None, :]
    s = xp @ pj.T
    cross = xa @ pj.T + xp @ aj.T
    db = xb[:, None, :] - bj[None, :, :]
    ddb = (d * db).sum(-1)
    gq = (g[:, :, None] * (-d * cross[:, :, None]
                           + s[:, :, None] * (db - d * ddb[:, :, None] / s2))).sum(1) / s2
    gp = g @ aj + ((g * ddb) @ pj) / s2
    return gq, gp


def bh_bruteforce(q, p, sigma, theta, kappa=3.0, leaf_cap=1, alpha=None, beta=None):
    """Barnes-Hut right-hand side (and, with alpha/beta, the backward-stage
    products) by the definition.  An approximated node k acts as n_k virtual
    points at its centre C_k (mean member position) carrying the mean
    momentum P_k / n_k (and the mean alpha, beta).  Returns a dict with v, a
    (forward), gq, gp (backward, if requested) and the counters pairs,
    monopoles, visits summed over targets."""
    q = np.asarray(q, np.float64)
    p = np.asarray(p, np.float64)
    n = q.shape[0]
    adj = alpha is not None
    if adj:
        alpha = np.asarray(alpha, np.float64)
        beta = np.asarray(beta, np.float64)
    s2 = sigma * sigma
    v = np.zeros((n, 3))
    a = np.zeros((n, 3))
    gq = np.zeros((n, 3))
    gp = np.zeros((n, 3))
    out = {"pairs": 0, "monopoles": 0, "visits": 0}
    nodes, kids, leaf = _tree(q, leaf_cap)
    if n == 0:
        out.update(v=v, a=a, gq=gq, gp=gp)
        return out
    cut2 = (kappa * sigma) ** 2
    stack = [((0, 0), np.arange(n))]
    while stack:
        key, idx = stack.pop()
        mem = np.asarray(nodes[key], dtype=np.int64)
        out["visits"] += len(idx)
        x = q[idx]
        lo, hi = q[mem].min(0), q[mem].max(0)
        C = q[mem].mean(0)
        P = p[mem].sum(0)
        nk = len(mem)
        g = np.maximum(lo - x, x - hi)
        gg = np.where(g > 0.0, g * g, 0.0)
        dmin2 = gg[:, 0] + gg[:, 1] + gg[:, 2]
        dc = x - C
        d2 = dc[:, 0] * dc[:, 0] + dc[:, 1] * dc[:, 1] + dc[:, 2] * dc[:, 2]
        side = float((hi - lo).max())
        far = dmin2 >= cut2
        mac = np.ones(len(idx), bool) if np.isinf(theta) else side * side < (theta * theta) * d2
        approx = (nk >= 2) & far & mac
        ia = idx[approx]
        if len(ia):
            out["monopoles"] += len(ia)
            d = q[ia] - C
            gv = np.exp(-(d * d).sum(1) / (2.0 * s2))
            v[ia] += gv[:, None] * P
            a[ia] += (gv * (p[ia] @ P))[:, None] * d / s2
            if adj:
                A, B = alpha[mem].sum(0), beta[mem].sum(0)
                tq, tp = _adjoint_pairs(q[ia], p[ia], alpha[ia], beta[ia], C[None], P[None] / nk,
                                        A[None] / nk, B[None] / nk, np.array([float(nk)]), sigma)
                gq[ia] += tq
                gp[ia] += tp
        io = idx[~approx]
        if len(io) == 0:
            continue
        if leaf[key]:
            out["pairs"] += len(io) * nk
            d = q[io][:, None, :] - q[mem][None, :, :]
            gv = np.exp(-(d * d).sum(-1) / (2.0 * s2))
            v[io] += gv @ p[mem]
            w = gv * (p[io] @ p[mem].T)
            a[io] += (w[:, :, None] * d).sum(1) / s2
            if adj:
                tq, tp = _adjoint_pairs(q[io], p[io], alpha[io], beta[io], q[mem], p[mem],
                                        alpha[mem], beta[mem], np.ones(nk), sigma)
                gq[io] += tq
                gp[io] += tp
        else:
            for c in kids[key]:
                stack.append((c, io))
    out.update(v=v, a=a, gq=gq, gp=gp)
    return out


def adjoint_vjp_torch(q, p, alpha, beta, sigma):
    """(dPhi/dq, dPhi/dp) for Phi = <alpha, v> + <beta, a>, (v, a) the exact
    right-hand side from float64 autograd of 1/2 <p, K(q) p>."""
    qt = torch.tensor(np.asarray(q, np.float64), requires_grad=True)
    pt = torch.tensor(np.asarray(p, np.float64), requires_grad=True)
    h = half_energy_torch(qt, pt, sigma)
    hq, hp = torch.autograd.grad(h, (qt, pt), create_graph=True)
    phi = (torch.tensor(np.asarray(alpha, np.float64)) * hp).sum() - (
        torch.tensor(np.asarray(beta, np.float64)) * hq).sum()
    gq, gp = torch.autograd.grad(phi, (qt, pt))
    return gq.numpy(), gp.numpy()
