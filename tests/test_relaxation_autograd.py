"""The relaxation-time bridge of autograd.py on the CPU: its forward value is
the library's decay fit and its backward pass applies the fit's
implicit-function weights, equal to the oracle's (needs no GPU: the fit is
host arithmetic in the library)."""
import numpy as np
import torch

from oracle import relaxation as rx
from paper_2511_09413_amd import autograd as ag


def test_relaxation_time_backward_is_the_oracle_weights():
    t0 = 1e-9
    t = np.linspace(t0, t0 + 20e-9, 200)
    m_np = rx.decay_model(t, t0, 0.3, 0.25, 4e-9) + np.random.default_rng(0).normal(0, 0.01, len(t))
    m = torch.tensor(m_np, requires_grad=True)
    tau = ag.relaxation_time(m, t, t0)
    ref, _ = rx.fit_decay(t, m_np, t0)
    assert abs(float(tau.detach()) - ref[2]) <= 1e-9 * ref[2]
    tau.backward(torch.tensor(2.5, dtype=torch.float64))
    w = rx.tau_weights(t, m_np, t0, ref)
    assert np.abs(m.grad.numpy() - 2.5 * w).max() <= 1e-8 * np.abs(2.5 * w).max()


def test_step_times():
    from workloads import Physics
    spec = ag.ObservableSpec(physics=Physics(), rails=[2], sites=[8], filling=[0.5], protocols=[([0.0], [0.0])],
                             n_steps=3)
    assert np.allclose(ag.step_times(spec), [1e-12, 2e-12, 3e-12])
