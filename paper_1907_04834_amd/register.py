"""Point-set registration by geodesic shooting (Sec. 2.1, eq. 2): the
initial momenta p0 that carry a template q0 onto a target minimise

    E(p0) = |q(1) - target|^2 / n + lam <p0, K(q0) p0>,

found with L-BFGS (as in Sec. 2.1).  Every objective and gradient is one call
of gs_shoot_adjoint (forward shooting with checkpoints, discrete adjoint) on
the device; this module only drives torch's L-BFGS.
"""
from __future__ import annotations

import torch

from . import gs


def register(q0, target, sigma, nt=40, lam=1e-4, method="exact", theta=0.5, leaf_cap=16,
             max_iter=50, p0=None, ckpt_every=8):
    """Returns (p0, history): the optimised float32 (n, 3) momenta and the
    objective after every evaluation."""
    if p0 is None:
        p0 = torch.zeros_like(q0)
    p = p0.detach().clone().requires_grad_(True)
    opt = torch.optim.LBFGS([p], lr=1.0, max_iter=max_iter, history_size=10,
                            line_search_fn="strong_wolfe", tolerance_grad=0.0,
                            tolerance_change=0.0)
    history = []

    def closure():
        opt.zero_grad()
        loss = gs.shoot_loss(p, q0, target, sigma, nt=nt, lam=lam, method=method, theta=theta,
                             leaf_cap=leaf_cap, ckpt_every=ckpt_every)
        loss.backward()
        history.append(float(loss))
        return loss

    opt.step(closure)
    return p.detach(), history
