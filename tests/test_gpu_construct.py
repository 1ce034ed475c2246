"""GPU parity of building a Fourier PlenOctree from per-frame PlenOctrees:
per-frame values carried onto the union leaves (bit-exact copies), the
per-leaf DFT against the FP64 reference, the bake -> DFT round trip, and the
whole construction against the oracle's construction, rendered."""
import numpy as np
import pytest

from oracle import dft
from paper_2202_08614_amd import _lib, construct, synth
from tests.gpu_util import check_parity, conditioned_reference, note, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _mixed_frames(seed, T, depth):
    rng = np.random.default_rng(seed)
    frames = []
    for f in range(T):
        leaves = synth.random_tree_leaves(seed * 100 + f, depth, p_split=0.5)
        frames.append(leaves[rng.random(len(leaves)) < 0.8])
    return frames


def _values(n, seed):
    """Snapshot records [n][32]: sigma, 27 SH coefficients, zero padding."""
    rng = np.random.default_rng(seed)
    v = np.zeros((n, 32), np.float32)
    v[:, 0] = np.maximum(rng.standard_normal(n) * 2.0, 0.0).astype(np.float32)
    v[:, 1:28] = rng.standard_normal((n, 27)).astype(np.float32)
    return v


def _dft_bound(vals, T):
    """(T + 4) u sum_t |x_t c_i b_i(t)| per output (u = 2^-24), plus
    5e-14 c sum_t |x_t| for the FP64 reference's own basis rounding (its phase
    i pi t / T < 31 pi carries up to 97 * 2^-52 = 2.2e-14): where
    i t is a multiple of T the exact basis value is 0, which the device's
    exact-phase sinpi returns and FP64 sin(k pi) misses by ~1e-16 k (with few
    frames whole columns alias to zero)."""
    B = np.stack([dft.basis(t, float(T), 31) for t in range(T)])
    c = np.full(31, 2.0 / T)
    c[0] = 1.0 / T
    a = np.abs(vals.astype(np.float64))
    ms = np.einsum("tl,ti->li", a[:, :, 0], (T + 4) * 2.0 ** -24 * np.abs(B) * c + 5e-14 * c)
    mz = np.einsum("tlq,ti->lqi", a[:, :, 1:28], (T + 4) * 2.0 ** -24 * np.abs(B[:, :5]) * c[:5] + 5e-14 * c[:5])
    return np.concatenate([ms, mz.reshape(a.shape[1], -1)], 1)


def test_frame_values_are_exact_copies(dev):
    import torch
    frames = _mixed_frames(3, 5, 5)
    union = _lib.union_leaves(np.concatenate(frames), 6)
    children, perm = _lib.build_tree(union, 6)
    slot_cells = union[perm]
    cells_d = torch.from_numpy(np.ascontiguousarray(slot_cells)).to(dev)
    n_bad = torch.zeros(1, dtype=torch.int32, device=dev)
    for t, f in enumerate(frames):
        vals = _values(len(f), 10 + t)
        ft = _lib.FrameTree(f, 6, dev)
        out = torch.full((len(union), 32), float("nan"), device=dev)
        note(f"fpo_frame_values frame {t}")
        _lib.frame_values(ft, torch.from_numpy(vals).to(dev), cells_d, out, n_bad)
        torch.cuda.synchronize()
        want = dft.frame_values_on_union(f, vals[:, :28], [tuple(c) for c in slot_cells])
        got = out.cpu().numpy()
        assert np.array_equal(got[:, :28], want.astype(np.float32))
        assert np.all(got[:, 28:] == 0.0)
    assert int(n_bad.item()) == 0


def test_frame_values_flag_cells_coarser_than_the_frame(dev):
    """A cell list that does not refine the frame is counted, and its cells get zeros."""
    import torch
    frame = np.array([[2, 0, 0, 0], [2, 1, 0, 0], [1, 1, 1, 1]], np.int32)
    cells = np.array([[1, 0, 0, 0], [1, 1, 1, 1], [2, 3, 3, 3]], np.int32)   # (1,0,0,0) is split in the frame
    ft = _lib.FrameTree(frame, 3, dev)
    vals = _values(3, 4)
    out = torch.full((3, 32), float("nan"), device=dev)
    n_bad = torch.zeros(1, dtype=torch.int32, device=dev)
    note("fpo_frame_values coarser cell")
    _lib.frame_values(ft, torch.from_numpy(vals).to(dev), torch.from_numpy(cells).to(dev), out, n_bad)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert int(n_bad.item()) == 1
    assert np.all(got[0] == 0.0)
    assert np.array_equal(got[1, :28], vals[2, :28]) and np.array_equal(got[2, :28], vals[2, :28])


@pytest.mark.parametrize("T", [60, 7])
@pytest.mark.parametrize("literal", [False, True])
def test_dft_matches_oracle(dev, T, literal):
    import torch
    L, stride = 333, 345
    rng = np.random.default_rng(T + 7 * literal)
    vals = np.zeros((T, stride, 32), np.float32)
    vals[:, :L, :28] = rng.standard_normal((T, L, 28)).astype(np.float32)
    note(f"fpo_dft_frames T={T} literal={literal}")
    coeffs, smax = _lib.dft_frames(torch.from_numpy(vals).to(dev), L, literal=literal)
    torch.cuda.synchronize()
    got = coeffs.cpu().numpy().reshape(stride, 192)
    want = dft.dft(vals[:, :L, :28], literal=literal)
    bound = _dft_bound(vals[:, :L], T)
    assert np.all(np.abs(got[:L, :166] - want) <= bound + 1e-30)
    assert np.all(got[:L, 166:] == 0.0)
    assert np.array_equal(smax.cpu().numpy()[:L], vals[:, :L, 0].max(0))


def test_bake_then_dft_round_trip(dev):
    """Baking a tree at t = 0 .. 59 and taking the DFT returns its coefficients."""
    import torch
    dijk = synth.random_tree_leaves(12, 6, p_split=0.6)
    k = synth.gaussian_coeffs(len(dijk), seed=12)
    tree = _lib.DeviceTree.from_leaves(dijk, k, 6, device=dev)
    basis = torch.from_numpy(_lib.time_basis([float(t) for t in range(60)])).to(dev)
    note("bake 60 times + fpo_dft_frames")
    snaps = _lib.bake_times(tree, basis, _lib.FPO_F32)
    coeffs, _ = _lib.dft_frames(snaps, tree.n_leaves)
    torch.cuda.synchronize()
    got = coeffs.cpu().numpy().reshape(tree.leaf_stride, 192)[:, :166]
    want = np.empty_like(got)
    want[:] = k[tree.perm]
    # bake error (32 terms) then DFT error (64 terms), both relative to sum |k b|
    mag = np.abs(k[tree.perm]).sum(1, keepdims=True)
    assert np.all(np.abs(got - want) <= 2.0 ** -15 * mag)


def test_construction_matches_oracle_and_renders(oracle_lib, dev):
    """Per-frame blob octrees (depth 6, 12 frames, mixed depths) -> union ->
    per-frame values -> DFT -> pruning, against the oracle's construction;
    then the built FPO renders within 1e-4 of the oracle's render of the
    oracle-built FPO."""
    import torch
    T = 12
    frames = synth.blob_frame_leaves(6, 8000, n_frames=T)
    vals = [_values(len(f), 100 + t) for t, f in enumerate(frames)]
    vals_d = [torch.from_numpy(v).to(dev) for v in vals]
    note("construct.build_fpo 12 frames depth 6")
    tree, leaves, info = construct.build_fpo(frames, vals_d, 6, dev)
    torch.cuda.synchronize()
    assert info["n_bad"] == 0
    U = dft.union_leaves(frames)
    assert info["union_leaves"] == len(U)
    per = np.stack([dft.frame_values_on_union(f, v[:, :28], U) for f, v in zip(frames, vals)])
    keep = dft.prune(U, per)
    assert info["kept"] == len(keep) < len(U)
    k_ref = dft.dft(per[:, keep])
    ref_leaves = np.array(U)[keep]
    # same leaf set
    assert set(map(tuple, leaves.tolist())) == set(map(tuple, ref_leaves.tolist()))
    # coefficients leaf by leaf
    pos = {tuple(c): i for i, c in enumerate(ref_leaves.tolist())}
    order = np.array([pos[tuple(c)] for c in leaves.tolist()])
    got = tree.coeffs.cpu().numpy().reshape(tree.leaf_stride, 192)[:tree.n_leaves, :166]
    got_caller = np.empty_like(got)
    got_caller[tree.perm] = got
    bound = _dft_bound(per[:, keep][:, order], T)
    assert np.all(np.abs(got_caller - k_ref[order]) <= bound + 1e-30)
    # render at a frame time and between frames
    cams = [synth.ring_camera(0.6 + j, 0.25, 1.5, 40.0, 56, 40, t) for j, t in enumerate((3.0, 7.5))]
    rgb, _ = _lib.render(tree, cams, _lib.make_opts(stop_T=1e-3))
    torch.cuda.synchronize()
    ot = oracle_lib.OracleTree(ref_leaves, 6)
    p = oracle_lib.make_params(period=float(T), stop_T=1e-3)
    for c, cam in enumerate(cams):
        o, d = oracle_lib.camera_rays(cam)
        ref = conditioned_reference(oracle_lib, ot, k_ref, p, [cam.time], o, d, np.zeros(len(o), np.int32))
        check_parity(rgb[c].cpu().numpy().reshape(-1, 3), ref, 1e-4)
