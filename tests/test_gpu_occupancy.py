"""GPU tests of the occupancy at one time: fpo_prune_at and
fpo_prune_at_sigma (per-time child tables in which subtrees without an opaque
leaf are empty, from snapshot records or the bake's density plane) and
fpo_coarse_occupancy_at (the dilated 64^3 grid over the leaves opaque at
that time).  Inputs that decide opacity are the oracle's bake, rounded to the
snapshot's precision, so the expected tables follow from the paper's Eq. 7
and the ReLU by a plain recursion; renders through the pruned tables are
checked against the oracle and against the unpruned render."""
import math

import copy

import numpy as np
import pytest

from oracle import codec, occupancy
from paper_2202_08614_amd import _lib, synth
from tests.gpu_util import check_parity, conditioned_reference, note, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _oracle_snapshots(oracle_lib, coeffs, times, perm, stride, dtype):
    """The oracle's bake [n_t][28][L] rounded to F32 or BF16, as snapshot
    records [n_t][stride][32] in slot order, plus the rounded values."""
    import torch
    vals = oracle_lib.bake(coeffs.astype(np.float64), oracle_lib.make_params(), times)       # [n_t][28][L]
    if dtype == _lib.FPO_F32:
        vals = vals.astype(np.float32).astype(np.float64)
        recs = np.zeros((len(times), stride, 32), np.float32)
        recs[:, :vals.shape[2], :28] = vals[:, :, perm].transpose(0, 2, 1)
        return torch.from_numpy(recs), vals
    vals = codec.bf16_decode(codec.bf16_encode(vals.astype(np.float32))).astype(np.float64)
    recs = np.zeros((len(times), stride, 32), np.uint16)
    recs[:, :vals.shape[2], :28] = codec.bf16_encode(vals[:, :, perm].transpose(0, 2, 1).astype(np.float32))
    return torch.from_numpy(recs.view(np.int16)).view(torch.bfloat16), vals


def _expected_pruned(children: np.ndarray, opaque_slot: np.ndarray) -> np.ndarray:
    """Child slots whose subtree holds an opaque leaf, by a bottom-up recursion
    over the table (nodes are numbered breadth first, children after parents)."""
    n = children.shape[0]
    has = np.zeros(n, bool)
    out = children.copy()
    for node in range(n - 1, -1, -1):
        for c in range(8):
            e = int(children[node, c])
            if e < 0:
                keep = bool(opaque_slot[-e - 1])
            elif e > 0:
                keep = bool(has[e])
            else:
                keep = False
            if not keep:
                out[node, c] = 0
            has[node] |= keep
    return out


@pytest.mark.parametrize("dtype", [_lib.FPO_F32, _lib.FPO_BF16])
def test_prune_and_occupancy_at_match_definitions(oracle_lib, dev, dtype):
    import torch
    dijk = synth.random_tree_leaves(31, 6, p_split=0.6)
    k = synth.gaussian_coeffs(len(dijk), seed=31)
    tree = _lib.DeviceTree.from_leaves(dijk, k, 6, device=dev, leaf_stride=len(dijk) + 5)
    times = [2.0, 19.5, 44.4]
    snaps, vals = _oracle_snapshots(oracle_lib, k, times, tree.perm, tree.leaf_stride, dtype)
    snaps = snaps.to(dev)
    note(f"fpo_prune_at / fpo_coarse_occupancy_at dtype={dtype}")
    pruned = _lib.prune_at(tree, snaps, dtype)
    cells = _lib.leaf_cells_slot_order(dijk, tree.perm, dev)
    bits = [_lib.coarse_occupancy_at(cells, 6, snaps[t], dtype, 64.0).cpu().numpy().view(np.uint32)
            for t in range(len(times))]
    torch.cuda.synchronize()
    children = tree.children.cpu().numpy()
    got = pruned.cpu().numpy()
    for t in range(len(times)):
        opaque_caller = vals[t, 0] > 0.0                       # sigma_scale 64 > 0: opaque iff sigma(t) > 0
        assert 0.2 < opaque_caller.mean() < 0.8
        opaque_slot = opaque_caller[tree.perm]
        want = _expected_pruned(children, opaque_slot)
        assert np.array_equal(got[t], want), int((got[t] != want).sum())
        assert (want != 0).sum() < (children != 0).sum()
        want_bits = occupancy.to_words(occupancy.dilated(dijk[opaque_caller]))
        assert np.array_equal(bits[t], want_bits), int(np.unpackbits((bits[t] ^ want_bits).view(np.uint8)).sum())


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_prune_level_passes_on_shallow_trees(oracle_lib, dev, depth):
    """Trees of depth 1 to 3 (no node pass at depth 1, one or two level
    passes above it): the tables pruned one level per pass and by passes over
    every row both equal the bottom-up definition."""
    import torch
    dijk = synth.random_tree_leaves(40 + depth, depth, p_split=0.7)
    k = synth.gaussian_coeffs(len(dijk), seed=40 + depth)
    tree = _lib.DeviceTree.from_leaves(dijk, k, depth, device=dev, leaf_stride=len(dijk) + 3)
    assert tree.levels is not None and len(tree.levels) == depth + 1
    flat = copy.copy(tree)
    flat.levels = None
    times = [3.0, 31.0, 47.5]
    snaps, vals = _oracle_snapshots(oracle_lib, k, times, tree.perm, tree.leaf_stride, _lib.FPO_F32)
    snaps = snaps.to(dev)
    children = tree.children.cpu().numpy()
    for tr in (tree, flat):
        note(f"fpo_prune_at depth={depth} level passes={tr.levels is not None}")
        got = _lib.prune_at(tr, snaps, _lib.FPO_F32)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        for t in range(len(times)):
            want = _expected_pruned(children, (vals[t, 0] > 0.0)[tree.perm])
            assert np.array_equal(got[t], want), (depth, t, int((got[t] != want).sum()))


@pytest.mark.parametrize("dtype", [_lib.FPO_F32, _lib.FPO_BF16])
def test_render_through_pruned_tables(oracle_lib, dev, dtype):
    """Snapshot renders through the pruned table of their time equal the
    unpruned renders (segments with positive optical depth are the same) and
    pass the oracle parity; the skip modes (coarse, and proposal with an
    untrained network) also accept the per-time grid."""
    import torch
    dijk = synth.blob_leaves(7, 40000)
    k = synth.gaussian_coeffs(len(dijk), seed=77)
    tree = _lib.DeviceTree.from_leaves(dijk, k, 7, device=dev)
    times = [7.0, 33.3]
    snaps, vals = _oracle_snapshots(oracle_lib, k, times, tree.perm, tree.leaf_stride, dtype)
    snaps = snaps.to(dev)
    cams = [synth.ring_camera(0.3 + 1.1 * j, math.radians(5 + 7 * j), 1.5, 30.0, 72, 40, times[j % 2])
            for j in range(4)]
    note(f"renders through pruned tables dtype={dtype}")
    pruned = _lib.prune_at(tree, snaps, dtype)
    cells = _lib.leaf_cells_slot_order(dijk, tree.perm, dev)
    ot = oracle_lib.OracleTree(dijk, 7)
    p = oracle_lib.make_params(stop_T=1e-3)
    ws = _lib.skip_workspace(1, 40, 72, dev)
    packed = _lib.mlp_pack(torch.from_numpy(synth.mlp_init(19)).to(dev))
    for j, cam in enumerate(cams):
        t = j % 2
        opts = _lib.make_opts(stop_T=1e-3, snapshot=snaps[t], snapshot_dtype=dtype)
        plain, _ = _lib.render(tree, [cam], opts)
        pt = _lib.tree_with_children(tree, pruned[t])
        got, _ = _lib.render(pt, [cam], opts)
        bits_t = _lib.coarse_occupancy_at(cells, 7, snaps[t], dtype, 64.0)
        skip = _lib.make_opts(stop_T=1e-3, snapshot=snaps[t], snapshot_dtype=dtype,
                              flags=_lib.FPO_RENDER_SKIP_COARSE, coarse_bits=bits_t, workspace=ws)
        got_skip, _ = _lib.render(pt, [cam], skip)
        prop = _lib.make_opts(stop_T=1e-3, snapshot=snaps[t], snapshot_dtype=dtype,
                              flags=_lib.FPO_RENDER_SKIP_PROPOSAL, coarse_bits=bits_t, proposal=packed,
                              workspace=ws)
        got_prop, _ = _lib.render(tree, [cam], prop)
        torch.cuda.synchronize()
        diff = (got - plain).abs().amax(-1).cpu().numpy().ravel()
        assert float(plain.max()) > 0.05
        assert (diff > 0).mean() <= 0.02 and diff.max() <= 2e-5, (float((diff > 0).mean()), float(diff.max()))
        o, d = oracle_lib.camera_rays(cam)
        ref = conditioned_reference(oracle_lib, ot, None, p, [times[t]], o, d, np.zeros(len(o), np.int32),
                                    snapshot=vals[t])
        check_parity(got.cpu().numpy().reshape(-1, 3), ref, 1e-4)
        check_parity(got_skip.cpu().numpy().reshape(-1, 3), ref, 1e-4)
        check_parity(got_prop.cpu().numpy().reshape(-1, 3), ref, 1e-4)


# (store, n_t): each bake kernel (per-frame FMA kernels below 4 times, MFMA
# tiles from 4 on, ragged 16-time tiles; F32, BF16 and FP8 stores) and the
# layout kernel
SIGMA_PLANE_CASES = [(_lib.FPO_F32, 1), (_lib.FPO_F32, 3), (_lib.FPO_F32, 10), (_lib.FPO_F32, 21),
                     (_lib.FPO_BF16, 2), (_lib.FPO_BF16, 5), (_lib.FPO_FP8_E4M3, 2), (_lib.FPO_FP8_E4M3, 17),
                     ("layout_21_11", 2), ("layout_11_5_fp8", 3)]


@pytest.mark.parametrize("store,n_t", SIGMA_PLANE_CASES)
@pytest.mark.parametrize("out_dtype", [_lib.FPO_F32, _lib.FPO_BF16])
def test_bake_sigma_plane_is_record_value(dev, store, n_t, out_dtype):
    """fpo_bake_times sigma_out holds value 0 of every record it writes, as
    FP32, bit for bit; slots past n_leaves are left alone."""
    import torch
    dijk = synth.random_tree_leaves(13, 6, p_split=0.6)
    n = len(dijk)
    if store == "layout_21_11":
        k = synth.gaussian_coeffs(n, seed=13, n_sigma=21, n_sh_fourier=11)
        tree = _lib.DeviceTree.from_leaves(dijk, k, 6, device=dev, leaf_stride=n + 7, n_sigma=21, n_sh_fourier=11)
        layout = _lib.make_layout(n_sigma=21)
    elif store == "layout_11_5_fp8":
        k = synth.gaussian_coeffs(n, seed=13, n_sigma=11)
        tree = _lib.DeviceTree.from_leaves(dijk, k, 6, device=dev, leaf_stride=n + 7, n_sigma=11)
        tree = _lib.quantize(tree, _lib.FPO_FP8_E4M3)
        layout = _lib.make_layout(n_sigma=11)
    else:
        k = synth.gaussian_coeffs(n, seed=13)
        tree = _lib.DeviceTree.from_leaves(dijk, k, 6, device=dev, leaf_stride=n + 7)
        if store != _lib.FPO_F32:
            tree = _lib.quantize(tree, store)
        layout = _lib.make_layout()
    times = [0.7 + i * 59.0 / n_t for i in range(n_t)]
    basis = torch.from_numpy(_lib.time_basis(times, layout)).to(dev)
    sigma = torch.full((n_t, tree.leaf_stride), float("nan"), dtype=torch.float32, device=dev)
    note(f"fpo_bake_times sigma_out store={store} n_t={n_t} out={out_dtype}")
    out = _lib.bake_times(tree, basis, out_dtype, sigma_out=sigma)
    torch.cuda.synchronize()
    rec0 = out[:, :n, 0].float().cpu().numpy()
    got = sigma.cpu().numpy()
    assert np.array_equal(got[:, :n].view(np.uint32), rec0.view(np.uint32))
    assert np.isnan(got[:, n:]).all()
    assert (rec0 > 0).any() and (rec0 <= 0).any()


def test_prune_at_sigma_equals_prune_at(dev):
    """Tables pruned from the density plane equal those pruned from the
    records (F32 and BF16 snapshots, 12 times of a depth-7 blob scene), and
    one node pass per tree level (the tree's level offsets) gives the tables
    of max_depth - 1 passes over every row."""
    import torch
    dijk = synth.blob_leaves(7, 40000)
    k = synth.gaussian_coeffs(len(dijk), seed=5)
    tree = _lib.DeviceTree.from_leaves(dijk, k, 7, device=dev, leaf_stride=len(dijk) + 9)
    times = [2.5 * i + 0.1 for i in range(12)]
    basis = torch.from_numpy(_lib.time_basis(times)).to(dev)
    flat = copy.copy(tree)
    flat.levels = None          # node passes over every row instead of one level per pass
    assert tree.levels is not None
    for dt in (_lib.FPO_F32, _lib.FPO_BF16):
        sigma = torch.empty((len(times), tree.leaf_stride), dtype=torch.float32, device=dev)
        note(f"fpo_prune_at_sigma against fpo_prune_at dtype={dt}")
        snaps = _lib.bake_times(tree, basis, dt, sigma_out=sigma)
        a = _lib.prune_at(tree, snaps, dt)
        b = _lib.prune_at_sigma(tree, sigma)
        c = _lib.prune_at_sigma(flat, sigma)
        d = _lib.prune_at(flat, snaps, dt)
        torch.cuda.synchronize()
        assert torch.equal(a, b) and torch.equal(b, c) and torch.equal(c, d)
        kept = (a != 0).sum().item() / (len(times) * (tree.children != 0).sum().item())
        assert 0.2 < kept < 0.95, kept


def _grandchild_reference(children: np.ndarray, rows: int) -> np.ndarray:
    """The two-level table from its definition: (c, children[c][b]) for
    internal c, else (c, 0)."""
    n = children.shape[0]
    out = np.zeros((rows, 8, 8, 2), np.int32)
    c = children[:rows]                                   # [rows][8]
    out[..., 0] = c[:, :, None]
    inner = (c > 0) & (c < n)
    out[..., 1] = np.where(inner[:, :, None], children[np.where(inner, c, 0)], 0)
    return out.reshape(rows, 64, 2)


def test_grandchild_tables_match_definition(dev):
    """fpo_grandchild_tables of the union table and of three pruned tables
    equal the definition; the rows cover exactly the nodes with an internal
    child (breadth-first numbering puts them first)."""
    import torch
    dijk = synth.blob_leaves(7, 40000)
    k = synth.gaussian_coeffs(len(dijk), seed=21)
    tree = _lib.DeviceTree.from_leaves(dijk, k, 7, device=dev)
    children = tree.children.cpu().numpy()
    depth = np.zeros(len(children), int)
    for i in range(len(children)):
        depth[children[i][children[i] > 0]] = depth[i] + 1
    assert np.all(np.diff(depth) >= 0)
    assert tree.upper() == int(np.nonzero((children > 0).any(1))[0][-1]) + 1 < len(children)
    times = [3.0, 31.5, 47.25]
    basis = torch.from_numpy(_lib.time_basis(times)).to(dev)
    sigma = torch.empty((3, tree.leaf_stride), dtype=torch.float32, device=dev)
    _lib.bake_times(tree, basis, _lib.FPO_F32, sigma_out=sigma)
    pruned = _lib.prune_at_sigma(tree, sigma)
    note("fpo_grandchild_tables union and 3 pruned tables")
    g_union = _lib.grandchild_tables(tree)
    g_pruned = _lib.grandchild_tables(tree, pruned)
    g_all = _lib.grandchild_tables(tree, n_rows=tree.n_nodes)
    torch.cuda.synchronize()
    rows = tree.upper()
    assert np.array_equal(g_union[0].cpu().numpy(), _grandchild_reference(children, rows))
    assert np.array_equal(g_all[0].cpu().numpy(), _grandchild_reference(children, tree.n_nodes))
    pr = pruned.cpu().numpy()
    for t in range(3):
        assert np.array_equal(g_pruned[t].cpu().numpy(), _grandchild_reference(pr[t], rows))


@pytest.mark.parametrize("dtype", [_lib.FPO_F32, _lib.FPO_BF16])
def test_renders_through_grandchild_tables_are_identical(dev, dtype):
    """Snapshot renders (plain, noalloc, coarse skip) through a view carrying
    a two-level table walk the same slots: the images equal those without it
    bit for bit, for the union table and for a pruned table, with the table
    over the upper nodes and over every node."""
    import torch
    dijk = synth.blob_leaves(7, 40000)
    k = synth.gaussian_coeffs(len(dijk), seed=23)
    tree = _lib.DeviceTree.from_leaves(dijk, k, 7, device=dev)
    times = [12.5]
    basis = torch.from_numpy(_lib.time_basis(times)).to(dev)
    sigma = torch.empty((1, tree.leaf_stride), dtype=torch.float32, device=dev)
    snap = _lib.bake_times(tree, basis, dtype, sigma_out=sigma)
    pruned = _lib.prune_at_sigma(tree, sigma)
    pt = _lib.tree_with_children(tree, pruned[0])
    cams = [synth.ring_camera(0.4 + 0.9 * j, math.radians(8 + 9 * j), 1.5, 30.0, 96, 64, times[0]) for j in range(4)]
    bits = torch.from_numpy(_lib.coarse_occupancy(dijk, 7).view(np.int32)).to(dev)
    ws = _lib.skip_workspace(4, 64, 96, dev)
    plain = _lib.make_opts(stop_T=1e-3, snapshot=snap[0], snapshot_dtype=dtype)
    skip = _lib.make_opts(stop_T=1e-3, snapshot=snap[0], snapshot_dtype=dtype, flags=_lib.FPO_RENDER_SKIP_COARSE,
                          coarse_bits=bits, workspace=ws)
    for base in (tree, pt):
        note(f"renders through grandchild tables dtype={dtype} pruned={base is pt}")
        for rows in (None, tree.n_nodes):
            g = _lib.grandchild_tables(tree, base.children, n_rows=rows)
            gt = _lib.tree_with_children(base, base.children, g[0])
            for opts in (plain, skip):
                want, _ = _lib.render(base, cams, opts)
                got, _ = _lib.render(gt, cams, opts)
                torch.cuda.synchronize()
                assert torch.equal(got, want)
            want, _ = _lib.render_noalloc(base, cams, plain)
            got, _ = _lib.render_noalloc(gt, cams, plain)
            torch.cuda.synchronize()
            assert torch.equal(got, want)
            assert float(want.max()) > 0.05


def test_c2_pruned_decode_sampled(oracle_lib, dev):
    """The pruned decode path at full size: the 2M-leaf scene, the step's 10
    times baked into F32 snapshots and pruned in one call each, 16 cameras of
    1080p per time through the pruned tables (the benchmark's launches); 3000
    sampled pixels of every launch against the oracle, and the images against
    the unpruned renders."""
    import torch
    sc = synth.c2_scene()
    tree = _lib.DeviceTree.from_leaves(sc.leaf_dijk, sc.coeffs, sc.max_depth, device=dev)
    cams = sc.cameras
    n_t, per = 10, 16
    times = [cams[j * per].time for j in range(n_t)]
    basis = torch.from_numpy(_lib.time_basis(times)).to(dev)
    note("c2 decode + prune at 10 times")
    sigma = torch.empty((n_t, tree.leaf_stride), dtype=torch.float32, device=dev)
    snap = _lib.bake_times(tree, basis, _lib.FPO_F32, sigma_out=sigma)
    pruned = _lib.prune_at_sigma(tree, sigma)
    assert torch.equal(pruned, _lib.prune_at(tree, snap, _lib.FPO_F32))
    torch.cuda.synchronize()
    kept = (pruned != 0).sum(dim=(1, 2)).cpu().numpy() / float((tree.children != 0).sum())
    assert np.all(kept < 0.95), kept
    gc = _lib.grandchild_tables(tree, pruned)
    ot = oracle_lib.OracleTree(sc.leaf_dijk, sc.max_depth)
    p = oracle_lib.make_params(stop_T=1e-3)
    rng = np.random.default_rng(10)
    for j in (0, 5, 9):
        opts = _lib.make_opts(stop_T=1e-3, snapshot=snap[j], snapshot_dtype=_lib.FPO_F32)
        note(f"c2 pruned render time index {j}")
        got, _ = _lib.render(_lib.tree_with_children(tree, pruned[j]), cams[j * per:(j + 1) * per], opts)
        plain, _ = _lib.render(tree, cams[j * per:(j + 1) * per], opts)
        two, _ = _lib.render(_lib.tree_with_children(tree, pruned[j], gc[j]), cams[j * per:(j + 1) * per], opts)
        torch.cuda.synchronize()
        assert torch.equal(two, got)
        diff = (got - plain).abs().amax(-1)
        assert float((diff > 0).float().mean()) <= 1e-3 and float(diff.max()) <= 2e-5
        m = 3000
        ci = rng.integers(0, per, m); py = rng.integers(0, 1080, m); px = rng.integers(0, 1920, m)
        vals = got[torch.from_numpy(ci).to(dev), torch.from_numpy(py).to(dev), torch.from_numpy(px).to(dev)]
        o = np.zeros((m, 3)); d = np.zeros((m, 3))
        for c in np.unique(ci):
            sel = np.nonzero(ci == c)[0]
            o[sel], d[sel] = oracle_lib.camera_rays(cams[j * per + c], px[sel], py[sel])
        ref = conditioned_reference(oracle_lib, ot, sc.coeffs, p, [times[j]], o, d, np.zeros(m, np.int32))
        check_parity(vals.cpu().numpy().astype(np.float64), ref, 1e-4)
