"""Pins for the reference proposal network and its labels."""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2202_08614_amd import synth


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    inp = np.concatenate([rng.uniform(0, 1, (n, 3)), rng.standard_normal((n, 3)), rng.uniform(0, 1, (n, 1))], 1)
    inp[:, 3:6] /= np.linalg.norm(inp[:, 3:6], axis=1, keepdims=True)
    lab = np.stack([rng.random(n) < 0.5, rng.uniform(0, 1, n), rng.uniform(0, 1, n)], 1).astype(np.float64)
    return inp, lab


def test_encoding_layout():
    x = np.array([[0.25, 0, 0, 0, 0, 0, 0.5]])
    g = mlp.encode(x)
    assert g.shape == (1, 84)
    # component 0, frequency 0: sin(pi/4), cos(pi/4); frequency 1: sin(pi/2) = 1
    assert np.allclose(g[0, 0:4], [np.sqrt(0.5), np.sqrt(0.5), 1.0, 0.0], atol=1e-15)
    # component 6 (t/T = 0.5), frequency 0: sin(pi/2) = 1, cos = 0
    assert np.allclose(g[0, 72:74], [1.0, 0.0], atol=1e-15)


def test_mlp_matches_torch_autograd():
    """Forward, loss and every weight gradient against torch autograd (FP64, CPU)."""
    w = mlp.init_weights(3)
    for k in ("b1", "b2", "b3"):
        w[k] = np.random.default_rng(4).standard_normal(w[k].shape) * 0.1
    inp, lab = _batch(97, 5)
    o, cache = mlp.forward(w, inp)
    loss, g_out = mlp.loss_and_grad_out(o, lab)
    grads = mlp.backward(w, cache, g_out)

    tw = {k: torch.tensor(v, requires_grad=True) for k, v in w.items()}
    g = torch.tensor(mlp.encode(inp))
    h = torch.relu(g @ tw["W1"] + tw["b1"])
    h = torch.relu(h @ tw["W2"] + tw["b2"])
    to = h @ tw["W3"] + tw["b3"]
    y = torch.tensor(lab)
    bce = torch.nn.functional.binary_cross_entropy_with_logits(to[:, 0], y[:, 0], reduction="none")
    tot = bce
    for j, q in ((1, 0.1), (2, 0.9)):
        u = y[:, j] - torch.sigmoid(to[:, j])
        tot = tot + torch.where(y[:, 0] > 0.5, torch.maximum(q * u, (q - 1) * u), torch.zeros_like(u))
    tl = tot.mean()
    tl.backward()
    assert np.allclose(o, to.detach().numpy(), atol=1e-12)
    assert abs(loss - float(tl.detach())) < 1e-12
    for k in w:
        assert np.allclose(grads[k], tw[k].grad.numpy(), atol=1e-12), k


def test_mlp_central_differences():
    w = mlp.init_weights(11)
    inp, lab = _batch(31, 12)
    o, cache = mlp.forward(w, inp)
    _, g_out = mlp.loss_and_grad_out(o, lab)
    grads = mlp.backward(w, cache, g_out)
    rng = np.random.default_rng(0)
    h = 1e-6
    for k in ("W1", "b1", "W2", "W3", "b3"):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in w[k].shape)
            wp = {kk: v.copy() for kk, v in w.items()}
            wm = {kk: v.copy() for kk, v in w.items()}
            wp[k][idx] += h
            wm[k][idx] -= h
            lp = mlp.loss_and_grad_out(mlp.forward(wp, inp)[0], lab)[0]
            lm = mlp.loss_and_grad_out(mlp.forward(wm, inp)[0], lab)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, grads[k][idx])


def test_labels_match_brute_force(oracle_lib):
    """hit / s_in / s_out from the oracle walk equal a direct scan of the
    brute-force segment list."""
    from oracle.brute import leaf_sigma_rgb, slab_segments
    depth = 4
    dijk = synth.random_tree_leaves(31, depth, p_split=0.6)
    k = synth.gaussian_coeffs(len(dijk), seed=31).astype(np.float64)
    tree = oracle_lib.OracleTree(dijk, depth)
    o, d = synth.random_rays(60, 32, inside_frac=0.1)
    o, d = o.astype(np.float64), d.astype(np.float64)
    times = [13.0]
    p = oracle_lib.make_params(sigma_scale=8.0, stop_T=1e-2)
    lab = oracle_lib.ray_labels(tree, k, p, times, o, d, np.zeros(60, np.int32))
    n_hit = 0
    for r in range(60):
        dd = d[r] / np.linalg.norm(d[r])
        idx, t0, t1 = slab_segments(dijk, o[r], dd)
        inp = mlp.ray_inputs(o[r:r + 1], d[r:r + 1], np.array([13.0]))
        T, first, last, hit = 1.0, None, None, False
        for l, a, b in zip(idx, t0, t1):
            s, _ = leaf_sigma_rgb(k[l], 13.0, dd, sigma_scale=8.0)
            if s * (b - a) > 0:
                first = a if first is None else first
                last = b
                hit = True
            T *= np.exp(-s * (b - a))
            if T < 1e-2:
                break
        assert lab[r, 0] == float(hit)
        if hit:
            n_hit += 1
            # chord through the cube from the entry point
            lo = np.max(np.minimum((0 - o[r]) / dd, (1 - o[r]) / dd))
            hi = np.min(np.maximum((0 - o[r]) / dd, (1 - o[r]) / dd))
            t_in = max(lo, 0.0)
            assert abs(lab[r, 1] - (first - t_in) / (hi - t_in)) < 1e-12
            assert abs(lab[r, 2] - (last - t_in) / (hi - t_in)) < 1e-12
            assert np.allclose(inp[0, :3], o[r] + t_in * dd)
    assert n_hit > 10


def test_flat_layout_round_trip_and_order():
    w = mlp.init_weights(5)
    w["b1"] = np.arange(64.0)
    p = mlp.to_flat(w)
    assert p.shape == (9795,)
    # row-major [85][64]: W1[k][j] at k*64 + j, b1 on row 84
    assert p[3 * 64 + 7] == w["W1"][3, 7]
    assert np.array_equal(p[84 * 64:85 * 64], np.arange(64.0))
    assert p[85 * 64 + 65 * 64 + 10 * 3 + 2] == w["W3"][10, 2]
    back = mlp.from_flat(p)
    for k in w:
        assert np.array_equal(back[k], w[k])


def test_fp16_forward_within_rounding_bound():
    """FP16 inference differs from the exact network by at most a few FP16
    roundings (2^-11 relative) of each propagated term; a transposed or
    misplaced operand would be off by O(magnitude)."""
    w = mlp.init_weights(8)
    for k in ("b1", "b2", "b3"):
        w[k] = np.random.default_rng(9).standard_normal(w[k].shape) * 0.2
    inp, _ = _batch(500, 10)
    exact, _ = mlp.forward(w, inp)
    half = mlp.forward_fp16(w, inp)
    mag = mlp.magnitude(w, inp)
    err = np.abs(half - exact)
    assert np.all(err <= 2.0 ** -8 * mag)
    assert err.max() > 0          # the rounding is really applied


def test_coarse_occupancy_against_box_overlap(oracle_lib):
    """The index-range definition against a continuous box-overlap test: cell
    (x, y, z) is set iff some leaf box meets the open block of the cell and its
    neighbours, [(x-1)/64, (x+2)/64) per axis."""
    from oracle import occupancy
    rng = np.random.default_rng(3)
    dijk = synth.random_tree_leaves(17, 7, p_split=0.5)[:300]
    dijk = np.vstack([dijk, [[3, 1, 6, 2]], [[2, 0, 0, 3]]])          # coarser-than-grid leaves
    grid = occupancy.dilated(dijk)
    lo = dijk[:, 1:4] / 2.0 ** dijk[:, :1]
    hi = (dijk[:, 1:4] + 1) / 2.0 ** dijk[:, :1]
    cells = rng.integers(0, 64, (3000, 3))
    cells = np.vstack([cells, np.argwhere(grid)[:, ::-1][rng.integers(0, grid.sum(), 500)]])
    for x, y, z in cells:
        blo = (np.array([x, y, z]) - 1) / 64.0
        bhi = (np.array([x, y, z]) + 2) / 64.0
        want = np.any(np.all((lo < bhi) & (blo < hi), axis=1))
        assert grid[z, y, x] == want, (x, y, z)
    assert 0 < grid.sum() < 64 ** 3
    words = occupancy.to_words(grid)
    idx = (5 * 64 + 9) * 64 + 33
    assert ((words[idx >> 5] >> (idx & 31)) & 1) == grid[5, 9, 33]
