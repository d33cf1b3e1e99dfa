"""The exact right-hand side that allocates nothing (gs_rhs_exact_static,
workspace in the library's static device array) against gs_rhs_exact, called
through the C ABI: two calls in a row, the second on a smaller point set, so
the second runs on an array that still holds the first call's contents."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1907_04834_amd import gs
from paper_1907_04834_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rel(x, y):
    x = x.detach().cpu().numpy().astype(np.float64)
    y = y.detach().cpu().numpy().astype(np.float64)
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def _static_call(q, p, prm):
    """Direct C-ABI call: the caller passes inputs and outputs only (the
    largest size, GS_STATIC_MAX_N, is one of the cases)."""
    dq, dp = torch.empty_like(q), torch.empty_like(q)
    L = gs.lib()
    st = L.gs_rhs_exact_static(ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(p.data_ptr()),
                               q.shape[0], ctypes.byref(prm), ctypes.c_void_p(dq.data_ptr()),
                               ctypes.c_void_p(dp.data_ptr()),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, L.gs_last_error().decode()
    return dq, dp


@pytest.mark.parametrize("sizes", [(20000, 5000), (500000, 1500)])
def test_static_workspace_matches_gs_rhs_exact(sizes):
    dev = torch.device("cuda:0")
    outs = []
    for n in sizes:
        print(f"gs_rhs_exact_static n={n}", flush=True)
        w = W.ellipsoid_20k(seed=7 + n, n=n)
        q = torch.from_numpy(w.q0).to(dev)
        p = torch.from_numpy(w.p0).to(dev)
        prm = gs.params(w.sigma)
        outs.append((_static_call(q, p, prm), gs.gs_rhs_exact(q, p, prm)))
    torch.cuda.synchronize()
    for (sq, sp), (eq, ep) in outs:
        # same kernels, at most a different FP64 chunking of the source sums
        assert _rel(sq, eq) < 1e-6 and _rel(sp, ep) < 1e-6
        assert torch.isfinite(sq).all() and torch.isfinite(sp).all()


def test_static_workspace_rejects_too_many_points():
    dev = torch.device("cuda:0")
    n = gs.GS_STATIC_MAX_N + 1
    q = torch.zeros((n, 3), dtype=torch.float32, device=dev)
    with pytest.raises(gs.GsError, match="GS_STATIC_MAX_N"):
        gs.gs_rhs_exact_static(q, q, gs.params(0.05))
