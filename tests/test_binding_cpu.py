"""CPU checks of the Python binding's argument marshalling: host tensors,
wrong dtypes and wrong shapes are refused before any library call (the
binding only marshals; the product path never computes on the CPU)."""
import numpy as np
import pytest
import torch

from paper_1907_04834_amd import gs


def _host(n=8, dtype=torch.float32):
    return torch.from_numpy(np.zeros((n, 3))).to(dtype)


@pytest.mark.parametrize("call", [
    lambda q, p, prm: gs.gs_rhs_exact(q, p, prm),
    lambda q, p, prm: gs.gs_rhs_bh(q, p, prm),
    lambda q, p, prm: gs.gs_shoot(q, p, prm, gs.GS_EXACT),
    lambda q, p, prm: gs.gs_shoot(q, p, prm, gs.GS_BH),
])
def test_host_tensors_are_refused(call):
    prm = gs.params(0.1, nt=2)
    with pytest.raises(TypeError, match="device tensor"):
        call(_host(), _host(), prm)


def test_f64_calls_refuse_host_tensors():
    prm = gs.params(0.1, nt=2)
    with pytest.raises(TypeError, match="device tensor"):
        gs.gs_rhs_exact_f64(_host(dtype=torch.float64), _host(dtype=torch.float64), prm)
    with pytest.raises(TypeError, match="device tensor"):
        gs.gs_shoot_f64(_host(dtype=torch.float64), _host(dtype=torch.float64), prm)


def test_non_tensor_inputs_are_refused():
    prm = gs.params(0.1, nt=2)
    with pytest.raises(TypeError):
        gs.gs_rhs_exact(np.zeros((8, 3), np.float32), np.zeros((8, 3), np.float32), prm)
