"""The runout + settlement objective of the differentiable column, on the
CPU: its value against hand-computed cases and its autograd gradient against
the closed form."""
import math

import numpy as np
import torch

from paper_2203_05562_amd.adjoint import runout_settlement


def test_objective_value_closed_form():
    # three points: horizontal distances 3, 4 (a 3-4-5 offset) and 1 from the axis at (1, 2)
    x0 = torch.tensor([[4.0, 2.0, 0.0], [1.0, 6.0, 1.0], [1.0, 3.0, 2.0]], dtype=torch.float64)
    u = torch.zeros_like(x0)
    u[2, 2] = -0.25                           # the top point settles by 0.25
    tau = 0.5
    J = runout_settlement(u, x0, [2], (1.0, 2.0), tau)
    R = tau * math.log(math.exp(3 / tau) + math.exp(4 / tau) + math.exp(1 / tau))
    assert abs(float(J) - (R + 0.25)) <= 1e-14 * R
    # tau -> 0 gives the largest distance
    J0 = runout_settlement(u, x0, [2], (1.0, 2.0), 1e-3)
    assert abs(float(J0) - (4.0 + 0.25)) <= 1e-12


def test_objective_gradient_closed_form():
    rng = np.random.default_rng(0)
    x0 = torch.tensor(rng.normal(size=(7, 3)), dtype=torch.float64)
    u = torch.tensor(rng.normal(size=(7, 3)) * 0.1, dtype=torch.float64, requires_grad=True)
    top, axis, tau = [1, 4, 5], (0.2, -0.1), 0.3
    J = runout_settlement(u, x0, top, axis, tau)
    J.backward()
    x = (x0 + u).detach().numpy()
    dx, dy = x[:, 0] - axis[0], x[:, 1] - axis[1]
    r = np.hypot(dx, dy)
    w = np.exp((r - r.max()) / tau)
    w /= w.sum()                              # softmax weights of the smooth maximum
    g = np.zeros((7, 3))
    g[:, 0] = w * dx / r
    g[:, 1] = w * dy / r
    g[top, 2] -= 1.0 / len(top)
    assert np.max(np.abs(u.grad.numpy() - g)) <= 1e-13
