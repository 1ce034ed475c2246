"""Pin for the reference Adam update: torch.optim.Adam (CPU) and the first-step closed form."""
import numpy as np
import torch

from oracle.optim import adam


def test_adam_matches_torch_cpu():
    rng = np.random.default_rng(0)
    p0 = rng.standard_normal(64)
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    q, m, v = p0.copy(), np.zeros(64), np.zeros(64)
    for step in range(1, 8):
        g = rng.standard_normal(64) * (0.1 if step % 2 else 3.0)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        q, m, v = adam(q, g, m, v, step, 1e-2)
        assert np.allclose(q, p.detach().numpy(), rtol=0, atol=1e-14)


def test_adam_first_step_closed_form():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p, m, v = adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.1)
    assert np.allclose(p, -0.1 * g / (np.abs(g) + 1e-8), atol=1e-15)
