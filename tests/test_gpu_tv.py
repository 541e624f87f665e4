"""GPU parity of tv_grad / tv_div (K and -K^T) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from tests.helpers import img_err, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2201_05497_amd as P
    return P


@pytest.mark.parametrize("shape", [(1, 128, 128), (96, 200, 200), (7, 13, 29), (1, 1, 5), (3, 1, 1)])
def test_grad_div(P, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.normal(size=shape).astype(np.float32)
    w = rng.normal(size=(3,) + shape).astype(np.float32)
    gx = P.tv_grad(torch.as_tensor(x, device="cuda")).cpu().numpy()
    dv = P.tv_div(torch.as_tensor(w, device="cuda")).cpu().numpy()
    want_g = oracle.grad(x.astype(np.float64))
    want_d = -oracle.grad_adjoint(w.astype(np.float64))
    eg, ed = img_err(gx, want_g), img_err(dv, want_d)
    report(f"tv {shape}", grad=eg, div=ed)
    assert eg <= 1e-6 and ed <= 1e-6
