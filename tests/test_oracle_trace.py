"""Pins for the oracle's octree point location and segment lists (DDA)."""
import numpy as np
import pytest

from oracle.brute import slab_segments
from paper_2202_08614_amd import synth


def _tree(oracle_lib, seed, depth):
    dijk = synth.random_tree_leaves(seed, depth)
    return dijk, oracle_lib.OracleTree(dijk, depth)


@pytest.mark.parametrize("seed,depth", [(0, 3), (1, 4), (2, 5)])
def test_locate_matches_box_scan(oracle_lib, seed, depth):
    dijk, tree = _tree(oracle_lib, seed, depth)
    G = 1 << depth
    rng = np.random.default_rng(seed)
    for _ in range(300):
        x, y, z = rng.integers(0, G, size=3)
        got = tree.locate(x, y, z)
        sh = depth - dijk[:, 0]
        hit = np.nonzero((dijk[:, 1] == (x >> sh)) & (dijk[:, 2] == (y >> sh)) & (dijk[:, 3] == (z >> sh)))[0]
        assert got == (int(hit[0]) if len(hit) else -1)


@pytest.mark.parametrize("seed,depth", [(0, 3), (1, 4), (2, 5), (3, 6)])
def test_trace_equals_brute_force(oracle_lib, seed, depth):
    """DDA + merge equals intersecting every leaf box and sorting (generic rays)."""
    dijk, tree = _tree(oracle_lib, seed, depth)
    o_all, d_all = synth.random_rays(200, seed + 100)
    n_nonempty = 0
    for o, d in zip(o_all.astype(np.float64), d_all.astype(np.float64)):
        leaf, t0, t1 = tree.trace(o, d)
        bl, b0, b1 = slab_segments(dijk, o, d)
        # the DDA merges touching cells of one leaf; brute force sees each leaf once
        assert list(leaf) == list(bl)
        assert np.allclose(t0, b0, atol=1e-12) and np.allclose(t1, b1, atol=1e-12)
        n_nonempty += len(leaf) > 0
    assert n_nonempty > 50


def test_trace_axis_aligned_and_corner_rays(oracle_lib):
    """Rays along an axis and through lattice corners (the tie cases)."""
    depth = 3
    dijk = np.array([[3, i, j, k] for i in range(8) for j in range(8) for k in range(8)
                     if (i + j + k) % 3 == 0], dtype=np.int32)
    tree = oracle_lib.OracleTree(dijk, depth)
    rays = [([-1.0, 0.3, 0.7], [1.0, 0.0, 0.0]),
            ([0.3, 2.0, 0.7], [0.0, -1.0, 0.0]),
            ([-0.5, -0.5, -0.5], [1.0, 1.0, 1.0]),          # through every lattice corner
            ([0.0, 0.0, 0.0], [1.0, 1.0, 0.0])]
    for o, d in rays:
        leaf, t0, t1 = tree.trace(np.array(o), np.array(d))
        bl, b0, b1 = slab_segments(dijk, o, d)
        keep = (b1 - b0) > 1e-12
        assert list(leaf) == list(bl[keep])
        assert np.all(t1 > t0)
        assert np.all(np.diff(t0) > 0)


def test_tree_validation(oracle_lib):
    ok = np.array([[1, 0, 0, 0], [2, 2, 0, 0]], dtype=np.int32)
    oracle_lib.OracleTree(ok, 3)
    bad = {
        1: np.array([[0, 0, 0, 0]], dtype=np.int32),          # depth 0
        2: np.array([[2, 4, 0, 0]], dtype=np.int32),          # outside the lattice
        3: np.array([[2, 1, 1, 1], [2, 1, 1, 1]], dtype=np.int32),
        4: np.array([[1, 0, 0, 0], [2, 1, 1, 1]], dtype=np.int32),  # (2,1,1,1) inside (1,0,0,0)
    }
    for code, dijk in bad.items():
        with pytest.raises(ValueError, match=f"error {code}"):
            oracle_lib.OracleTree(dijk, 3)
