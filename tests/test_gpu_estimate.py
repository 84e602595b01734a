"""GPU: likelihood-based estimation of theta = (log q1, log q2, log sigma)
through the autograd binding: L-BFGS on the pseudo-log-likelihood of
Section 5.1 with the nominal recomputed by IPLS at every evaluation and the
frozen-nominal gradient."""
import numpy as np
import pytest
import torch

from paper_2207_00426_amd import estimate, pss
from paper_2207_00426_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_lbfgs_improves_the_objective_and_sigma(dtype):
    w = wl.ct_batch(B=8, n=1500, seed=21, M=5)
    b = pss.Batch.ct(w.y_off, w.model, dtype=dtype, device="cuda")
    y = pss.to_soa(w.y, dtype, "cuda")
    th_true = np.array(w.model.theta)
    th0 = th_true + 0.5
    fit = estimate.fit_theta_lbfgs(b, y, th0, n_steps=20, passes=5)
    th = np.array(fit["theta"])
    assert np.isfinite(th).all() and np.isfinite(fit["loss_trace"]).all()
    assert fit["iterations"] >= 5 and fit["evaluations"] >= fit["iterations"]
    assert all(b <= a for a, b in zip(fit["loss_trace"], fit["loss_trace"][1:]))
    assert fit["loss_final"] < fit["loss_start"] - 0.1
    # the bearing noise is pinned down well by the data
    assert abs(th[2] - th_true[2]) < 0.1 < abs(th0[2] - th_true[2])
