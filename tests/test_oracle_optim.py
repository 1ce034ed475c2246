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


def test_adam_touched_matches_torch_sparse_adam():
    """Lazy Adam over records: torch.optim.SparseAdam with row-sparse
    gradients (whole records present or absent) updates exactly the present
    rows, moments included, with the global step count.  SparseAdam adds eps
    to sqrt(v) instead of sqrt(v_hat) (the paper's alternative form), so eps is
    taken negligible here, where the two forms coincide."""
    from oracle.optim import adam_touched
    rng = np.random.default_rng(1)
    n_rec, rec = 40, 8
    p0 = rng.standard_normal((n_rec, rec))
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.SparseAdam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-30)
    q, m, v = p0.ravel().copy(), np.zeros(n_rec * rec), np.zeros(n_rec * rec)
    for step in range(1, 8):
        rows = np.sort(rng.choice(n_rec, 13, replace=False))
        g = np.zeros((n_rec, rec))
        g[rows] = rng.standard_normal((13, rec)) * (0.1 if step % 2 else 3.0)
        g[rows[0], :] = 0.0
        g[rows[0], 3] = 0.5           # a touched record that is zero but for one value
        opt.zero_grad()
        p.grad = torch.sparse_coo_tensor(torch.tensor(rows)[None], torch.tensor(g[rows]), (n_rec, rec))
        opt.step()
        q, m, v = adam_touched(q, g.ravel(), m, v, step, 1e-2, rec, eps=1e-30)
        assert np.allclose(q, p.detach().numpy().ravel(), rtol=0, atol=1e-14)
        assert np.allclose(m, opt.state[p]["exp_avg"].numpy().ravel(), rtol=0, atol=1e-15)
    # a record with no gradient keeps its value and moments
    z = np.zeros(n_rec * rec)
    q2, m2, v2 = adam_touched(p0.ravel(), z, z + 0.3, z + 0.2, 3, 1e-2, rec)
    assert np.array_equal(q2, p0.ravel()) and np.all(m2 == 0.3) and np.all(v2 == 0.2)
