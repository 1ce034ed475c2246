"""GPU parity of the fine-tuning path (Sec. 4.3): backward against the FP64
oracle gradient and against central differences of the GPU forward, the L2
loss, the fused Adam step, and a short synthetic fine-tune."""
import numpy as np
import pytest

from oracle.optim import adam as adam_ref
from paper_2202_08614_amd import _lib, synth
from tests.gpu_util import check_parity, conditioned_reference, note, perpendicular_pair, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _unpack(recs: np.ndarray, perm: np.ndarray, n: int) -> np.ndarray:
    """[stride][48][4] F32 leaf records -> [L][166] caller order."""
    flat = recs.reshape(recs.shape[0], -1)[:n, :166]
    out = np.zeros_like(flat)
    out[perm] = flat
    return out


def _scene_and_rays(oracle_lib, n_rays, seed, depth=5):
    dijk = synth.shell_leaves(depth, 0.33, 0.09)
    coeffs = synth.gaussian_coeffs(len(dijk), seed=seed)
    cams = [synth.ring_camera(0.5 + 1.1 * k, 0.25 - 0.2 * k, 1.5, 40.0, 48, 48, 0.0) for k in range(3)]
    rng = np.random.default_rng(seed)
    ci = rng.integers(0, 3, n_rays)
    py = rng.integers(0, 48, n_rays)
    px = rng.integers(0, 48, n_rays)
    o = np.zeros((n_rays, 3)); d = np.zeros((n_rays, 3))
    for c in range(3):
        sel = np.nonzero(ci == c)[0]
        o[sel], d[sel] = oracle_lib.camera_rays(cams[c], px[sel], py[sel])
    times = [3.3, 27.1, 51.9]
    t_idx = rng.integers(0, 3, n_rays).astype(np.int32)
    return dijk, coeffs, o.astype(np.float32), d.astype(np.float32), times, t_idx


# forward: 4096 rays run one ray per wave, 40000 rays one ray per lane
@pytest.mark.parametrize("n_rays", [4096, 40000])
@pytest.mark.parametrize("stop_T", [0.0, 1e-2])
def test_backward_matches_oracle_gradient(oracle_lib, dev, stop_T, n_rays):
    import torch
    dijk, coeffs, o, d, times, t_idx = _scene_and_rays(oracle_lib, n_rays, 3)
    tree = _lib.DeviceTree.from_leaves(dijk, coeffs, 5, device=dev, sigma_scale=16.0)
    rng = np.random.default_rng(7)
    g_rgb = rng.standard_normal((len(o), 3)).astype(np.float32)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    basis = to(_lib.time_basis(times))
    opts = _lib.make_opts(stop_T=stop_T, bg=(0.2, 0.3, 0.4))
    note(f"backward vs oracle stop_T={stop_T} n_rays={n_rays}")
    rgb, _ = _lib.render_rays(tree, to(o), to(d), to(t_idx), basis, opts)
    grad = torch.zeros_like(tree.coeffs)
    _lib.render_backward(tree, to(o), to(d), to(t_idx), basis, rgb, to(g_rgb), grad, opts)
    torch.cuda.synchronize()
    got = _unpack(grad.cpu().numpy(), tree.perm, len(dijk))
    ot = oracle_lib.OracleTree(dijk, 5)
    p = oracle_lib.make_params(stop_T=stop_T, bg=(0.2, 0.3, 0.4), sigma_scale=16.0)
    want, rgb_ref = oracle_lib.render_grad(ot, coeffs, p, times, o.astype(np.float64), d.astype(np.float64),
                                           t_idx, g_rgb.astype(np.float64))
    gmax = np.abs(want).max()
    assert gmax > 0 and (np.abs(want) > 1e-3 * gmax).sum() > 1000
    bad = np.abs(got - want) > 1e-3 * np.abs(want) + 1e-5 * gmax
    assert not bad.any(), (bad.sum(), np.abs(got - want).max(), gmax)


# cap 1: nearly every ray overflows and is walked again; 4: a mix; 1000: every ray recorded
@pytest.mark.parametrize("cap", [1, 4, 1000])
@pytest.mark.parametrize("stop_T", [0.0, 1e-2])
def test_recorded_backward_matches_oracle_gradient(oracle_lib, dev, stop_T, cap):
    """FPO_RAYS_RECORD: the forward writes each ray's segments of positive
    optical depth; its colours equal the plain forward's bit for bit, its
    counts equal the oracle's opaque-segment counts (-1 where they exceed cap),
    and the backward from the records gives the plain backward's gradient (up
    to the order of the atomic additions) and the oracle's."""
    import torch
    n_rays = 4096
    dijk, coeffs, o, d, times, t_idx = _scene_and_rays(oracle_lib, n_rays, 3)
    tree = _lib.DeviceTree.from_leaves(dijk, coeffs, 5, device=dev, sigma_scale=16.0)
    rng = np.random.default_rng(7)
    g_rgb = rng.standard_normal((n_rays, 3)).astype(np.float32)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    o_d, d_d, t_d, g_d = to(o), to(d), to(t_idx), to(g_rgb)
    basis = to(_lib.time_basis(times))
    ws = _lib.record_workspace(n_rays, cap, dev)
    ws.fill_(-7)
    plain = _lib.make_opts(stop_T=stop_T, bg=(0.2, 0.3, 0.4))
    rec = _lib.make_opts(stop_T=stop_T, bg=(0.2, 0.3, 0.4), flags=_lib.FPO_RAYS_RECORD, workspace=ws)
    note(f"recorded backward stop_T={stop_T} cap={cap}")
    rgb0, _ = _lib.render_rays(tree, o_d, d_d, t_d, basis, plain)
    rgb1, _ = _lib.render_rays(tree, o_d, d_d, t_d, basis, rec)
    g0 = torch.zeros_like(tree.coeffs)
    g1 = torch.zeros_like(tree.coeffs)
    _lib.render_backward(tree, o_d, d_d, t_d, basis, rgb0, g_d, g0, plain)
    _lib.render_backward(tree, o_d, d_d, t_d, basis, rgb1, g_d, g1, rec)
    torch.cuda.synchronize()
    assert torch.equal(rgb0, rgb1)
    cnt = _lib.record_counts(ws, n_rays).cpu().numpy()
    ot = oracle_lib.OracleTree(dijk, 5)
    p = oracle_lib.make_params(stop_T=stop_T, bg=(0.2, 0.3, 0.4), sigma_scale=16.0)
    ref = oracle_lib.render_rays(ot, coeffs, p, times, o.astype(np.float64), d.astype(np.float64), t_idx)
    n_opq = ref["n_opaque"][:, 0]
    want_cnt = np.where(n_opq > cap, -1, n_opq)
    assert (cnt >= -1).all() and (cnt <= cap).all()
    assert (cnt == want_cnt).mean() >= 0.999, np.nonzero(cnt != want_cnt)[0][:10]
    assert ((cnt == -1).sum() > 0) == (n_opq.max() > cap)
    a = _unpack(g0.cpu().numpy(), tree.perm, len(dijk))
    b = _unpack(g1.cpu().numpy(), tree.perm, len(dijk))
    gmax = np.abs(a).max()
    assert gmax > 0 and np.all(np.abs(a - b) <= 1e-5 * np.abs(a) + 1e-7 * gmax), np.abs(a - b).max()
    want, _ = oracle_lib.render_grad(ot, coeffs, p, times, o.astype(np.float64), d.astype(np.float64),
                                     t_idx, g_rgb.astype(np.float64))
    bad = np.abs(b - want) > 1e-3 * np.abs(want) + 1e-5 * np.abs(want).max()
    assert not bad.any(), (bad.sum(), np.abs(b - want).max())


def test_two_level_table_gives_the_same_forward_and_backward(oracle_lib, dev):
    """Forward (one ray per wave, with segment records; one ray per lane) and
    backward (from the records; re-walking) through a view that carries the
    two-level table walk the same segments: colours, transmittance and
    records equal the plain view's bit for bit, gradients up to the order of
    the atomic additions."""
    import torch
    n_rays = 4096
    dijk = synth.blob_leaves(7, 30000)
    coeffs = synth.gaussian_coeffs(len(dijk), seed=17)
    tree = _lib.DeviceTree.from_leaves(dijk, coeffs, 7, device=dev, sigma_scale=16.0)
    two = _lib.tree_with_children(tree, tree.children, _lib.grandchild_tables(tree)[0])
    cams = [synth.ring_camera(0.5 + 1.7 * k, 0.2 - 0.15 * k, 1.5, 30.0, 64, 64, 0.0) for k in range(3)]
    rng = np.random.default_rng(17)
    ci = rng.integers(0, 3, n_rays)
    o = np.zeros((n_rays, 3)); d = np.zeros((n_rays, 3))
    for c in range(3):
        sel = np.nonzero(ci == c)[0]
        o[sel], d[sel] = oracle_lib.camera_rays(cams[c], rng.integers(0, 64, len(sel)), rng.integers(0, 64, len(sel)))
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    o_d, d_d = to(o.astype(np.float32)), to(d.astype(np.float32))
    t_d = to(rng.integers(0, 3, n_rays).astype(np.int32))
    g_d = to(rng.standard_normal((n_rays, 3)).astype(np.float32))
    basis = to(_lib.time_basis([4.0, 22.5, 40.1]))
    for n, flags in ((n_rays, _lib.FPO_RAYS_RECORD), (n_rays, 0), (40000, 0)):
        note(f"two-level table forward/backward n={n} flags={flags}")
        if n != n_rays:
            idx = torch.from_numpy(rng.integers(0, n_rays, n)).to(dev)
            oo, dd, tt, gg = o_d[idx].contiguous(), d_d[idx].contiguous(), t_d[idx].contiguous(), g_d[idx].contiguous()
        else:
            oo, dd, tt, gg = o_d, d_d, t_d, g_d
        out = {}
        for name, tr in (("plain", tree), ("two", two)):
            ws = _lib.record_workspace(n, 128, dev) if flags else None
            opts = _lib.make_opts(stop_T=1e-3, flags=flags, workspace=ws)
            rgb, T = _lib.render_rays(tr, oo, dd, tt, basis, opts, want_T=True)
            g = torch.zeros_like(tree.coeffs)
            if n <= 32768:
                _lib.render_backward(tr, oo, dd, tt, basis, rgb, gg, g, opts)
            torch.cuda.synchronize()
            out[name] = (rgb, T, g, None if ws is None else ws.clone())
        a, b = out["plain"], out["two"]
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        assert float(a[1].min()) < 0.5
        if a[3] is not None:
            assert torch.equal(_lib.record_counts(a[3], n), _lib.record_counts(b[3], n))
        if n <= 32768:
            ga, gb = a[2].cpu().numpy(), b[2].cpu().numpy()
            gmax = np.abs(ga).max()
            assert gmax > 0 and np.all(np.abs(ga - gb) <= 1e-5 * np.abs(ga) + 1e-7 * gmax)


def test_backward_matches_gpu_central_differences(oracle_lib, dev):
    """dL/dk on 64 coefficients against central differences (h = 1e-3) of
    the GPU forward, L = sum_r w_r . rgb_r accumulated in FP64."""
    import torch
    dijk, coeffs, o, d, times, t_idx = _scene_and_rays(oracle_lib, 2048, 5)
    tree = _lib.DeviceTree.from_leaves(dijk, coeffs, 5, device=dev, sigma_scale=16.0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    o_d, d_d, t_d = to(o), to(d), to(t_idx)
    basis = to(_lib.time_basis(times))
    w = np.random.default_rng(1).standard_normal((len(o), 3))
    w_d = to(w.astype(np.float32))
    opts = _lib.make_opts()
    note("backward vs GPU central differences")
    rgb, _ = _lib.render_rays(tree, o_d, d_d, t_d, basis, opts)
    grad = torch.zeros_like(tree.coeffs)
    _lib.render_backward(tree, o_d, d_d, t_d, basis, rgb, w_d, grad, opts)
    g = grad.cpu().numpy()
    rng = np.random.default_rng(2)
    flat = np.abs(g).reshape(-1)
    cand = np.nonzero(flat > 0.05 * flat.max())[0]
    assert len(cand) >= 64
    pick = rng.choice(cand, 64, replace=False)
    h = 1e-3
    flat_coeffs = tree.coeffs.view(-1)

    def loss():
        r, _ = _lib.render_rays(tree, o_d, d_d, t_d, basis, opts)
        return float((r.double().cpu().numpy() * w).sum())

    for idx in pick:
        k0 = float(flat_coeffs[idx])
        flat_coeffs[idx] = k0 + h
        lp = loss()
        flat_coeffs[idx] = k0 - h
        lm = loss()
        flat_coeffs[idx] = k0
        fd = (lp - lm) / (2 * h)
        an = float(g.reshape(-1)[idx])
        assert abs(fd - an) <= 2e-2 * abs(an) + 2e-3 * flat.max(), (idx, fd, an)


def test_l2_loss_kernel(dev):
    import torch
    rng = np.random.default_rng(4)
    imgs = rng.random((5, 7, 9, 3)).astype(np.float32)
    n = 1000
    ii, yy, xx = rng.integers(0, 5, n), rng.integers(0, 7, n), rng.integers(0, 9, n)
    rgb = rng.random((n, 3)).astype(np.float32)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    note("fpo_l2_loss")
    grad, loss = _lib.l2_loss(to(rgb), to(imgs), to(ii.astype(np.int32)), to(yy.astype(np.int32)),
                              to(xx.astype(np.int32)))
    torch.cuda.synchronize()
    tgt = imgs[ii, yy, xx].astype(np.float64)
    e = rgb.astype(np.float64) - tgt
    assert abs(float(loss.item()) - (e ** 2).sum() / n) < 1e-5
    assert np.allclose(grad.cpu().numpy(), 2 * e / n, atol=1e-7)


def test_adam_kernel_matches_reference(dev):
    import torch
    rng = np.random.default_rng(5)
    n = 4 * 10007
    p0 = rng.standard_normal(n).astype(np.float32)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    p, m, v = to(p0), torch.zeros(n, device=dev), torch.zeros(n, device=dev)
    q, mq, vq = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    scale = np.zeros(n)          # moving average of |g|: bounds the magnitude of every term in m
    note("fpo_adam_step")
    for step in range(1, 6):
        g0 = (rng.standard_normal(n) * 10.0 ** rng.integers(-4, 2, n)).astype(np.float32)
        g = to(g0)
        _lib.adam_step(p, g, m, v, step, lr=1e-2)
        # the kernel receives its hyperparameters as FP32 values; compare like with like
        q, mq, vq = adam_ref(q, g0, mq, vq, step, float(np.float32(1e-2)), float(np.float32(0.9)),
                             float(np.float32(0.999)), float(np.float32(1e-8)))
        scale = 0.9 * scale + 0.1 * np.abs(g0.astype(np.float64))
        torch.cuda.synchronize()
        assert float(g.abs().max()) == 0.0                # gradient cleared
        assert np.allclose(p.cpu().numpy(), q, rtol=1e-5, atol=1e-6)
        # two FP32 roundings per step, accumulated over the steps so far
        mg = m.cpu().numpy()
        ratio = np.abs(mg - mq) / (2 * step * 2.0 ** -23 * scale + 1e-30)
        k = int(np.argmax(ratio))
        assert ratio[k] <= 1.0, (step, k, float(mg[k]), float(mq[k]), float(g0[k]), float(scale[k]))


@pytest.mark.parametrize("device_step", [False, True])
def test_adam_touched_matches_reference(dev, device_step):
    """fpo_adam_step_touched against the lazy-Adam reference: records of 192
    floats, a third of them with an all-zero gradient each step (one record
    zero but for its last value); untouched records keep parameters and
    moments bit for bit, touched ones follow Adam with the global step."""
    import torch
    from oracle.optim import adam_touched
    rng = np.random.default_rng(6)
    n_rec, rec = 3001, 192
    n = n_rec * rec
    p0 = rng.standard_normal(n).astype(np.float32)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    p, m, v = to(p0), torch.zeros(n, device=dev), torch.zeros(n, device=dev)
    state = torch.zeros(4, dtype=torch.int32, device=dev) if device_step else None
    q, mq, vq = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    scale = np.zeros(n)          # moving average of |g|: bounds the magnitude of every term in m
    f32 = lambda x: float(np.float32(x))
    note(f"fpo_adam_step_touched device_step={device_step}")
    for step in range(1, 5):
        g0 = (rng.standard_normal((n_rec, rec)) * 10.0 ** rng.integers(-3, 1, (n_rec, 1))).astype(np.float32)
        g0[rng.random(n_rec) < 1 / 3] = 0.0
        g0[7] = 0.0
        g0[7, rec - 1] = 0.25
        p_before, m_before, v_before = p.clone(), m.clone(), v.clone()
        g = to(g0.ravel())
        _lib.adam_step_touched(p, g, m, v, step=0 if device_step else step, lr=1e-2, state=state)
        q, mq, vq = adam_touched(q, g0.ravel(), mq, vq, step, f32(1e-2), rec, f32(0.9), f32(0.999), f32(1e-8))
        hit = np.repeat(np.any(g0 != 0, axis=1), rec)
        scale[hit] = 0.9 * scale[hit] + 0.1 * np.abs(g0.ravel()[hit].astype(np.float64))
        torch.cuda.synchronize()
        assert float(g.abs().max()) == 0.0
        untouched = torch.from_numpy(~np.any(g0 != 0, axis=1)).to(dev).repeat_interleave(rec)
        assert untouched.any() and not untouched.all()
        for now, before in ((p, p_before), (m, m_before), (v, v_before)):
            assert torch.equal(now[untouched], before[untouched])
        assert np.allclose(p.cpu().numpy(), q, rtol=1e-5, atol=1e-6)
        # two FP32 roundings per step, accumulated over the steps so far
        assert np.all(np.abs(m.cpu().numpy() - mq) <= 2 * step * 2.0 ** -23 * scale + 1e-30)
        if device_step:
            assert int(state[0]) == step


def test_finetune_converges(dev):
    """A small fine-tune: targets rendered from a ground-truth tree, start from
    GT + N(0, 0.05) noise, 8192-ray batches, L2 loss, Adam; the loss falls."""
    import torch
    from paper_2202_08614_amd.finetune import FineTuner
    dijk = synth.blob_leaves(6, 6000, n_frames=8)
    gt = synth.gaussian_coeffs(len(dijk), seed=1)
    init = synth.perturb_coeffs(gt, 0.05, seed=2)
    cams = [synth.ring_camera(2 * np.pi * k / 6, 0.26, 1.5, 30.0, 96, 96, t) for t in (1.0, 31.0) for k in range(6)]
    note("fine-tune 60 steps")
    ft = FineTuner.from_scene(dijk, gt, init, 6, cams, dev, sigma_scale=64.0, stop_T=1e-3, lr=1e-2,
                              batch=8192, seed=3)
    first = ft.train(5)
    ft.train(50)
    last = ft.train(5)
    torch.cuda.synchronize()
    assert np.mean(last) < 0.5 * np.mean(first), (first, last)


@pytest.fixture(scope="module")
def c4(dev):
    sc = synth.c4_scene()
    tree = _lib.DeviceTree.from_leaves(sc.leaf_dijk, sc.coeffs, sc.max_depth, device=dev)
    return sc, tree


def test_c4_batch_gradient_matches_oracle(oracle_lib, dev, c4):
    """The fine-tune step at full size: the 500k-leaf depth-8 scene, one
    8192-ray batch drawn over its 24 cameras x 30 times at 800x800 (the
    benchmark's batch); forward colours and the gradient of every coefficient
    against the FP64 oracle.  Colours go through the parity check (ties
    exempt by their FP64 spread under a 2e-7 sideways shift, the placement
    error of an FP32 camera ray).  The gradient gets the same rule per
    coefficient: its FP64 spread is the largest change of the oracle's
    gradient when every ray of the batch moves sideways by 2e-7; a
    coefficient whose spread exceeds the bar is a tie and must stay within
    its spread at 1e-6 plus the bar.  Leaves crossed by a ray whose early
    termination straddles the threshold (the two sides may stop after
    different segments) and density coefficients of leaves whose density sum
    sits at the ReLU kink within FP32 rounding are exempt too; together the
    exempt coefficients are at most 1% of the nonzero ones (about 0.3% here:
    a 2e-7 shift moves the segment lengths of grazing crossings by more than
    the 1e-3 relative gradient bar, while the colours barely move)."""
    import torch
    sc, tree = c4
    cams = sc.cameras
    times = sorted({c.time for c in cams})
    ci, py, px = synth.sample_pixels(8192, len(cams), 800, 800)
    o = np.zeros((8192, 3)); d = np.zeros((8192, 3))
    for c in np.unique(ci):
        sel = np.nonzero(ci == c)[0]
        o[sel], d[sel] = oracle_lib.camera_rays(cams[c], px[sel], py[sel])
    t_idx = np.array([times.index(cams[c].time) for c in ci], np.int32)
    g_rgb = np.random.default_rng(8).standard_normal((8192, 3)).astype(np.float32)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    basis = to(_lib.time_basis(times))
    ws = _lib.record_workspace(8192, 128, dev)
    plain = _lib.make_opts(stop_T=1e-3)
    rec = _lib.make_opts(stop_T=1e-3, flags=_lib.FPO_RAYS_RECORD, workspace=ws)
    ot = oracle_lib.OracleTree(sc.leaf_dijk, sc.max_depth)
    p = oracle_lib.make_params(stop_T=1e-3)
    g64 = g_rgb.astype(np.float64)
    want, rgb_ref = oracle_lib.render_grad(ot, sc.coeffs, p, times, o, d, t_idx, g64)
    ref = conditioned_reference(oracle_lib, ot, sc.coeffs, oracle_lib.make_params(stop_T=1e-3, band=1e-3), times,
                                o, d, t_idx)
    gmax = np.abs(want).max()
    assert gmax > 0 and (np.abs(want) > 1e-3 * gmax).sum() > 10000
    bar = 1e-3 * np.abs(want) + 1e-5 * gmax
    # the gradient's FP64 spread under sideways shifts of every ray
    u, v = perpendicular_pair(d)
    gspread = {}
    for eps in (2e-7, 1e-6):
        sp = np.zeros_like(want)
        for sgn, w in ((1.0, u), (-1.0, u), (1.0, v), (-1.0, v)):
            alt, _ = oracle_lib.render_grad(ot, sc.coeffs, p, times, o + sgn * eps * w, d, t_idx, g64)
            sp = np.maximum(sp, np.abs(alt - want))
        gspread[eps] = sp
    tie = gspread[2e-7] > bar
    # leaves of rays whose early termination straddles the threshold within the FP32 accuracy of
    # the transmittance (a relative 1e-4: some 10 segments of FP32 exp and optical depth)
    near = oracle_lib.render_rays(ot, sc.coeffs, oracle_lib.make_params(stop_T=1e-3, band=1e-4), times, o, d,
                                  t_idx, n_threads=8)["rgb"]
    straddle = np.nonzero(np.abs(near[:, 0] - near[:, 1]).max(axis=1) > 0)[0]
    touched = set()
    for r in straddle:
        touched.update(int(x) for x in ot.trace(o[r], d[r])[0])
    exempt = tie.copy()
    if touched:
        exempt[np.array(sorted(touched))] = True
    # ReLU kinks: where a crossed leaf's density sum sigma_raw(t) lies within FP32 rounding of 0
    # (|sigma_raw| <= 2^-18 sum_i |k_i b_i|, four times the 31-term bound), FP32 and FP64 may
    # take different sides of the ReLU and the derivative of the density coefficients jumps by
    # s b_i dL/dsigma (the derivative at the kink is 0); the colour is continuous there
    kink = set()
    B = np.stack([oracle_lib.basis(t, 60.0, 31) for t in times])
    for ti in range(len(times)):
        leaves = set()
        for r in np.nonzero(t_idx == ti)[0]:
            leaves.update(int(x) for x in ot.trace(o[r], d[r])[0])
        if not leaves:
            continue
        lv = np.array(sorted(leaves), np.int64)
        sraw = sc.coeffs[lv, :31].astype(np.float64) @ B[ti]
        mag = np.abs(sc.coeffs[lv, :31].astype(np.float64)) @ np.abs(B[ti])
        kink.update(int(x) for x in lv[np.abs(sraw) <= 2.0 ** -18 * mag])
    if kink:
        exempt[np.array(sorted(kink)), :31] = True
    assert exempt.sum() <= 1e-2 * (want != 0).sum(), (int(exempt.sum()), int((want != 0).sum()))
    # the plain backward (rays walked again) and the one from segment records (as the fine-tune runs)
    for name, opts in (("plain", plain), ("recorded", rec)):
        note(f"c4 render_rays + render_backward ({name}) 8192 rays, 500k leaves")
        rgb, _ = _lib.render_rays(tree, to(o.astype(np.float32)), to(d.astype(np.float32)), to(t_idx), basis,
                                  opts)
        grad = torch.zeros_like(tree.coeffs)
        _lib.render_backward(tree, to(o.astype(np.float32)), to(d.astype(np.float32)), to(t_idx), basis, rgb,
                             to(g_rgb), grad, opts)
        torch.cuda.synchronize()
        got = _unpack(grad.cpu().numpy(), tree.perm, sc.n_leaves)
        check_parity(rgb.cpu().numpy(), ref)
        err = np.abs(got - want)
        bad = err > bar
        assert not (bad & ~exempt).any(), (name, int((bad & ~exempt).sum()), err[~exempt].max(), gmax)
        assert not (tie & (err > gspread[1e-6] + bar)).any(), (name, "a tie coefficient beyond its 1e-6 spread")
        print(f"[c4 {name}] gradient ties {int(tie.sum())} coefficients, straddle rays {len(straddle)} "
              f"({len(touched)} leaves), ReLU-kink leaves {len(kink)}; off the bar {int(bad.sum())}, all exempt")
    assert (_lib.record_counts(ws, 8192) >= 0).all()


def test_c4_backward_matches_central_differences(oracle_lib, dev, c4):
    """The check the fine-tune configuration names, at its size: on the 500k-leaf
    scene and one 8192-ray batch, dL/dk from the recorded forward and the
    backward from segment records (as the fine-tuner runs them) on 64
    coefficients against central differences (h = 1e-3) of the GPU forward,
    L = sum_r w_r . rgb_r accumulated in FP64.  Without early termination:
    a perturbation that moves a ray's transmittance across the threshold
    changes its colour by a step, which no derivative describes."""
    import torch
    sc, tree = c4
    cams = sc.cameras
    times = sorted({c.time for c in cams})
    ci, py, px = synth.sample_pixels(8192, len(cams), 800, 800)
    o = np.zeros((8192, 3)); d = np.zeros((8192, 3))
    for c in np.unique(ci):
        sel = np.nonzero(ci == c)[0]
        o[sel], d[sel] = oracle_lib.camera_rays(cams[c], px[sel], py[sel])
    t_idx = np.array([times.index(cams[c].time) for c in ci], np.int32)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    o_d, d_d, t_d = to(o.astype(np.float32)), to(d.astype(np.float32)), to(t_idx)
    basis = to(_lib.time_basis(times))
    w = np.random.default_rng(11).standard_normal((8192, 3))
    ws = _lib.record_workspace(8192, 128, dev)
    opts = _lib.make_opts(stop_T=0.0, flags=_lib.FPO_RAYS_RECORD, workspace=ws)
    plain = _lib.make_opts(stop_T=0.0)
    note("c4 recorded backward vs GPU central differences, 64 coefficients")
    rgb, _ = _lib.render_rays(tree, o_d, d_d, t_d, basis, opts)
    grad = torch.zeros_like(tree.coeffs)
    _lib.render_backward(tree, o_d, d_d, t_d, basis, rgb, to(w.astype(np.float32)), grad, opts)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().reshape(-1)
    flat_abs = np.abs(g)
    cand = np.nonzero(flat_abs > 0.05 * flat_abs.max())[0]
    assert len(cand) >= 64
    pick = np.random.default_rng(12).choice(cand, 64, replace=False)
    h = 1e-3
    flat_coeffs = tree.coeffs.view(-1)

    def loss():
        r, _ = _lib.render_rays(tree, o_d, d_d, t_d, basis, plain)
        return float((r.double().cpu().numpy() * w).sum())

    for idx in pick:
        k0 = float(flat_coeffs[idx])
        flat_coeffs[idx] = k0 + h
        lp = loss()
        flat_coeffs[idx] = k0 - h
        lm = loss()
        flat_coeffs[idx] = k0
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[idx]) <= 2e-2 * abs(g[idx]) + 2e-3 * flat_abs.max(), (int(idx), fd, float(g[idx]))


@pytest.mark.parametrize("n_rays", [1, 32768])
def test_recorded_path_at_its_limits(oracle_lib, dev, n_rays):
    """FPO_RAYS_RECORD at one ray and at the largest batch it accepts (32768,
    the last one-ray-per-wave batch): the recording forward's colours equal the
    plain forward's, and the gradient from the records equals the re-walk's up
    to the order of the atomic additions."""
    import torch
    dijk, coeffs, o, d, times, t_idx = _scene_and_rays(oracle_lib, max(n_rays, 2), 17)
    o, d, t_idx = o[:n_rays], d[:n_rays], t_idx[:n_rays]
    tree = _lib.DeviceTree.from_leaves(dijk, coeffs, 5, device=dev, sigma_scale=16.0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    o_d, d_d, t_d = to(o), to(d), to(t_idx)
    if n_rays == 1:     # a ray through the shell, so that the single ray has segments
        o_d = to(np.array([[0.5, 0.5, -0.5]], np.float32))
        d_d = to(np.array([[0.013, 0.021, 1.0]], np.float32))
    g_d = to(np.random.default_rng(5).standard_normal((n_rays, 3)).astype(np.float32))
    basis = to(_lib.time_basis(times))
    ws = _lib.record_workspace(n_rays, 64, dev)
    plain = _lib.make_opts(stop_T=1e-3)
    rec = _lib.make_opts(stop_T=1e-3, flags=_lib.FPO_RAYS_RECORD, workspace=ws)
    note(f"recorded path n_rays={n_rays}")
    rgb0, _ = _lib.render_rays(tree, o_d, d_d, t_d, basis, plain)
    rgb1, _ = _lib.render_rays(tree, o_d, d_d, t_d, basis, rec)
    g0 = torch.zeros_like(tree.coeffs)
    g1 = torch.zeros_like(tree.coeffs)
    _lib.render_backward(tree, o_d, d_d, t_d, basis, rgb0, g_d, g0, plain)
    _lib.render_backward(tree, o_d, d_d, t_d, basis, rgb1, g_d, g1, rec)
    torch.cuda.synchronize()
    assert torch.equal(rgb0, rgb1)
    cnt = _lib.record_counts(ws, n_rays).cpu().numpy()
    assert (cnt >= -1).all() and (cnt > 0).any()
    a, b = g0.cpu().numpy(), g1.cpu().numpy()
    gmax = np.abs(a).max()
    assert gmax > 0 and np.all(np.abs(a - b) <= 1e-5 * np.abs(a) + 1e-7 * gmax)


def test_finetune_graph_replays_match_eager_steps(dev):
    """The fine-tune step captured once in a HIP graph and replayed against the
    eager step on the same batches, with other GPU work and a synchronisation
    between the replays: after every step the moments agree, the parameters
    agree wherever the gradient's sign is not at the mercy of the order of the
    FP32 atomic additions (Adam's first steps move a parameter by lr times the
    sign of its gradient), the gradient is cleared, the device step count has
    advanced by one with the bias corrections of that step, and the losses
    agree."""
    import torch
    from paper_2202_08614_amd.finetune import FineTuner
    dijk = synth.blob_leaves(6, 6000, n_frames=8)
    gt = synth.gaussian_coeffs(len(dijk), seed=1)
    init = synth.perturb_coeffs(gt, 0.05, seed=2)
    cams = [synth.ring_camera(2 * np.pi * k / 6, 0.26, 1.5, 30.0, 96, 96, t) for t in (1.0, 31.0) for k in range(6)]
    note("fine-tune eager steps vs HIP graph replays")
    fe = FineTuner.from_scene(dijk, gt, init, 6, cams, dev, batch=8192, seed=3)
    fg = FineTuner.from_scene(dijk, gt, init, 6, cams, dev, batch=8192, seed=3, graph=True)
    le = torch.zeros(5, device=dev)
    lg = torch.zeros(5, device=dev)
    for k in range(5):
        b = fe.sample()
        fe.step(*b[:3], le[k:k + 1], t_idx=b[3])
        fg.step(*b[:3], lg[k:k + 1], t_idx=b[3])
        junk = torch.randn(1 << 16, device=dev).square().sum()      # other work between the replays
        torch.cuda.synchronize()
        assert float(junk) > 0
        assert int(fg.adam_state[0]) == k + 1
        c = fg.adam_state[1:3].view(torch.float32).cpu().numpy()
        t = k + 1
        b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))    # the betas reach the library as FP32
        assert np.allclose(c, [1 / (1 - b1 ** t), 1 / (1 - b2 ** t)], rtol=1e-6)
        assert not fg.grad.any() and not fe.grad.any()
        for a, b_ in ((fe.m, fg.m), (fe.v, fg.v)):
            scale = float(a.abs().max())
            assert scale > 0 and float((a - b_).abs().max()) <= 1e-4 * scale
        steady = fe.m.abs() > 1e-3 * float(fe.m.abs().max())
        assert int(steady.sum()) > 1000
        assert torch.allclose(fe.tree.coeffs[steady], fg.tree.coeffs[steady], rtol=1e-5, atol=1e-5)
    assert torch.allclose(le, lg, rtol=1e-4)


@pytest.mark.parametrize("graph", [False, True])
def test_finetune_checkpoint_resume(dev, tmp_path, graph):
    """N steps in one run equal N/2 steps, save, a fresh fine-tuner loading the
    file, and N/2 more: the coefficients and Adam's moments agree (up to the
    order of the backward's FP32 atomic additions), the step count and the
    batch sampler continue where they stopped."""
    import torch
    from paper_2202_08614_amd.finetune import FineTuner
    dijk = synth.blob_leaves(6, 6000, n_frames=8)
    gt = synth.gaussian_coeffs(len(dijk), seed=1)
    init = synth.perturb_coeffs(gt, 0.05, seed=2)
    cams = [synth.ring_camera(2 * np.pi * k / 6, 0.26, 1.5, 30.0, 96, 96, t) for t in (1.0, 31.0) for k in range(6)]
    note(f"fine-tune checkpoint/resume graph={graph}")
    n = 6
    full = FineTuner.from_scene(dijk, gt, init, 6, cams, dev, batch=4096, seed=3, graph=graph)
    lf = torch.zeros(n, device=dev)
    for k in range(n):
        b = full.sample()
        full.step(*b[:3], lf[k:k + 1], t_idx=b[3])
    first = FineTuner.from_scene(dijk, gt, init, 6, cams, dev, batch=4096, seed=3, graph=graph)
    lh = torch.zeros(n, device=dev)
    for k in range(n // 2):
        b = first.sample()
        first.step(*b[:3], lh[k:k + 1], t_idx=b[3])
    path = str(tmp_path / "ft.pt")
    first.save(path)
    del first
    second = FineTuner.from_scene(dijk, gt, gt, 6, cams, dev, batch=4096, seed=99, graph=graph)   # other state
    second.load(path)
    assert second.t == n // 2
    for k in range(n // 2, n):
        b = second.sample()
        second.step(*b[:3], lh[k:k + 1], t_idx=b[3])
    torch.cuda.synchronize()
    assert second.t == n
    if graph:
        assert int(second.adam_state[0]) == n and int(full.adam_state[0]) == n
    for a, b_ in ((full.m, second.m), (full.v, second.v)):
        scale = float(a.abs().max())
        assert scale > 0 and float((a - b_).abs().max()) <= 1e-4 * scale
    steady = full.m.abs() > 1e-3 * float(full.m.abs().max())
    assert int(steady.sum()) > 1000
    assert torch.allclose(full.tree.coeffs[steady], second.tree.coeffs[steady], rtol=1e-5, atol=1e-5)
    assert torch.allclose(lf, lh, rtol=1e-4)
    # the sampler continues identically
    nb_f, nb_s = full.sample(), second.sample()
    assert all(torch.equal(x, y) for x, y in zip(nb_f, nb_s))
