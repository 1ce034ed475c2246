"""Pins for the oracle's PlenOctree fusion (Sec. 3, Eq. 3-5).

Closed cases: a first observation replaces the leaf values (W = 0), the
weight is the running mean of the transmittances (Eq. 5), Eq. 3 with that
weight after two and three views computed by hand, the transmittance of a
leaf behind another from the slab chord, the stop at tau, length weighting
within one view, and the walk's final transmittance against the oracle
render of the same values (a separately pinned path)."""
import math

import numpy as np
import pytest

from oracle import fusion
from oracle.brute import chord_length, leaf_boxes
from paper_2202_08614_amd import synth

S = 16.0      # sigma_scale


def _field(mu=((0.5, 0.5, 0.5),), w=(0.2,), a=(0.7,), seed=3):
    rng = np.random.default_rng(seed)
    return synth.Field(mu=np.array(mu, dtype=np.float64), w=np.array(w, dtype=np.float64),
                       a=np.array(a, dtype=np.float64), u=rng.normal(0, 1, (3, 3)), v=rng.normal(0, 1, (3, 3)),
                       b=rng.normal(0, 0.5, 3))


def test_field_closed_forms():
    f = _field(mu=((0.3, 0.4, 0.5), (5.0, 5.0, 5.0)), w=(0.1, 0.1), a=(0.8, 0.6))
    # at the first centre, the second Gaussian (50 widths away) adds nothing measurable
    assert abs(fusion.field_sigma(f, [0.3, 0.4, 0.5]) - 0.8) < 1e-12
    # one width away along x: a exp(-1/2)
    assert abs(fusion.field_sigma(f, [0.4, 0.4, 0.5]) - 0.8 * math.exp(-0.5)) < 1e-12
    g = synth.Field(mu=f.mu, w=f.w, a=f.a, u=np.zeros((3, 3)), v=np.zeros((3, 3)), b=np.array([0.0, 1.0, -2.0]))
    c = fusion.field_colour(g, [0.1, 0.2, 0.3], [0.0, 0.0, 1.0])
    assert np.allclose(c, [0.5, 1 / (1 + math.exp(-1.0)), 1 / (1 + math.exp(2.0))], atol=1e-15)


def _one_leaf():
    dijk = np.array([[2, 1, 2, 1]], dtype=np.int32)
    return dijk


def test_first_observation_replaces_values(oracle_lib):
    """W = C = 0: Eq. 3 gives sigma = sigma_obs, Eq. 4 z = Y(d) c(d), Eq. 5 W = T, C = 1."""
    dijk = _one_leaf()
    tree = oracle_lib.OracleTree(dijk, 3)
    f = _field()
    lo, hi = leaf_boxes(dijk)
    target = lo[0] + np.array([0.3, 0.6, 0.45]) * (hi[0] - lo[0])
    o = target + np.array([-1.3, 0.4, 0.2])
    d = target - o
    dn = d / np.linalg.norm(d)
    vals = np.zeros((1, 28))
    vals[0, 0] = 0.4
    acc, near, _ = fusion.observe_rays(oracle_lib, tree, vals, o, d, f, S, 1e-3)
    v, w, c = fusion.apply_view(vals, np.zeros(1), np.zeros(1, np.int64), acc)
    # the chord from the slab test, its midpoint and the field there
    L = chord_length(lo[0], hi[0], o, d)
    t_in = max(min((lo[0][a] - o[a]) / dn[a], (hi[0][a] - o[a]) / dn[a]) for a in range(3))
    x = o + (t_in + 0.5 * L) * dn
    assert abs(acc[0, 29] - L) < 1e-13
    assert abs(v[0, 0] - fusion.field_sigma(f, x)) < 1e-12
    Y = oracle_lib.sh9(dn)
    col = fusion.field_colour(f, x, dn)
    assert np.allclose(v[0, 1:28], np.outer(col, Y).reshape(-1), atol=1e-12)
    assert w[0] == pytest.approx(1.0, abs=1e-15) and c[0] == 1
    assert not near.any()


def _two_in_a_row():
    # two leaves along x at the same (y, z) cell: [0, 1/4) and [1/2, 3/4) in x
    return np.array([[2, 0, 1, 1], [2, 2, 1, 1]], dtype=np.int32)


def test_transmittance_behind_a_leaf(oracle_lib):
    """The second leaf is entered with T = exp(-s sigma_0 L_0); that is its
    weight after one view (W = 0 before)."""
    dijk = _two_in_a_row()
    tree = oracle_lib.OracleTree(dijk, 3)
    f = _field()
    o = np.array([-1.0, 0.37, 0.41])
    d = np.array([1.0, 0.013, -0.007])
    vals = np.zeros((2, 28))
    vals[0, 0] = 0.3
    vals[1, 0] = 5.0
    acc, _, T_end = fusion.observe_rays(oracle_lib, tree, vals, o, d, f, S, 1e-3)
    _, w, c = fusion.apply_view(vals, np.zeros(2), np.zeros(2, np.int64), acc)
    lo, hi = leaf_boxes(dijk)
    L0 = chord_length(lo[0], hi[0], o, d)
    L1 = chord_length(lo[1], hi[1], o, d)
    T1 = math.exp(-S * 0.3 * L0)
    assert w[0] == pytest.approx(1.0, abs=1e-15)
    assert abs(w[1] - T1) < 1e-13 and c.tolist() == [1, 1]
    assert abs(T_end[0] - T1 * math.exp(-S * 5.0 * L1)) < 1e-13


def test_stop_at_tau(oracle_lib):
    """A leaf entered with T <= tau is not observed: its values, W and C stay."""
    dijk = _two_in_a_row()
    tree = oracle_lib.OracleTree(dijk, 3)
    f = _field()
    o = np.array([-1.0, 0.37, 0.41])
    d = np.array([1.0, 0.0, 0.0])
    vals = np.zeros((2, 28))
    vals[0, 0] = 3.0          # optical depth 16 * 3 / 4 = 12: T = 6e-6 < 1e-3
    vals[1, 1:] = 0.25
    acc, _, T_end = fusion.observe_rays(oracle_lib, tree, vals, o, d, f, S, 1e-3)
    v, w, c = fusion.apply_view(vals, np.full(2, 0.7), np.array([3, 3]), acc)
    assert acc[1].tolist() == [0.0] * 30
    assert c.tolist() == [4, 3] and w[1] == 0.7 and np.array_equal(v[1], vals[1])
    assert abs(T_end[0] - math.exp(-12.0)) < 1e-15
    # with tau = 0 the second leaf is observed, with weight T = exp(-12)
    acc0, _, _ = fusion.observe_rays(oracle_lib, tree, vals, o, d, f, S, 0.0)
    assert abs(acc0[1, 0] / acc0[1, 29] - math.exp(-12.0)) < 1e-15


def test_three_views_by_hand(oracle_lib):
    """Views of one leaf with T = 1 and observed densities s1, s2, s3:
    W_1 = 1, sigma_1 = s1;  W_2 = 1, sigma_2 = (s1 + s2) / 2;
    sigma_3 = (W_2 sigma_2 + s3) / (W_2 + 1) = ((s1 + s2) / 2 + s3) / 2 (Eq. 3
    with the running-mean weight of Eq. 5, not the mean of three)."""
    dijk = _one_leaf()
    tree = oracle_lib.OracleTree(dijk, 3)
    f = _field(mu=((0.35, 0.6, 0.3),), w=(0.15,), a=(0.9,))
    lo, hi = leaf_boxes(dijk)
    centre = 0.5 * (lo[0] + hi[0])
    dirs = [np.array([1.0, 0.1, 0.05]), np.array([0.1, -1.0, 0.2]), np.array([-0.2, 0.15, 1.0])]
    offs = [np.array([0.0, 0.03, -0.02]), np.array([0.04, 0.0, 0.01]), np.array([-0.03, 0.02, 0.0])]
    vals = np.zeros((1, 28))
    W = np.zeros(1)
    C = np.zeros(1, np.int64)
    obs = []
    for dd, off in zip(dirs, offs):
        o = centre + off - 2.0 * dd
        acc, _, _ = fusion.observe_rays(oracle_lib, tree, vals, o, dd, f, S, 1e-3)
        obs.append(acc[0, 1] / acc[0, 0])           # sigma at this view's midpoint
        vals, W, C = fusion.apply_view(vals, W, C, acc)
    s1, s2, s3 = obs
    assert len({round(x, 9) for x in obs}) == 3
    assert abs(vals[0, 0] - ((s1 + s2) / 2 + s3) / 2) < 1e-13
    assert W[0] == pytest.approx(1.0, abs=1e-15) and C[0] == 3


def test_weight_is_running_mean(oracle_lib):
    """Eq. 5: after views with transmittances T_1..T_n, W = mean(T_i).  The
    leaf sits behind a first leaf whose density changes between views."""
    dijk = _two_in_a_row()
    tree = oracle_lib.OracleTree(dijk, 3)
    f = _field()
    o = np.array([-1.0, 0.37, 0.41])
    d = np.array([1.0, 0.0, 0.0])
    W = np.zeros(2)
    C = np.zeros(2, np.int64)
    Ts = []
    for s0 in (0.0, 0.2, 0.05, 0.4):
        vals = np.zeros((2, 28))
        vals[0, 0] = s0
        acc, _, _ = fusion.observe_rays(oracle_lib, tree, vals, o, d, f, S, 1e-3)
        Ts.append(math.exp(-S * s0 * 0.25))
        _, W, C = fusion.apply_view(vals, W, C, acc)
    assert abs(W[1] - np.mean(Ts)) < 1e-14 and C[1] == 4


def test_length_weighting_within_a_view(oracle_lib):
    """Two rays through one leaf in one view, T = 1 on both: the update
    uses the chord-weighted mean of the two midpoint densities."""
    dijk = _one_leaf()
    tree = oracle_lib.OracleTree(dijk, 3)
    f = _field(mu=((0.3, 0.6, 0.3),), w=(0.12,), a=(0.9,))
    lo, hi = leaf_boxes(dijk)
    # the first ray clips a corner of the leaf, the second crosses it along y
    o = np.array([[-1.0, 0.3, 0.3], [0.26, -1.0, 0.3]])
    d = np.array([[1.0, 0.35, 0.0], [0.12, 1.0, 0.0]])
    vals = np.zeros((1, 28))
    acc, _, _ = fusion.observe_rays(oracle_lib, tree, vals, o, d, f, S, 1e-3)
    v, w, _ = fusion.apply_view(vals, np.zeros(1), np.zeros(1, np.int64), acc)
    Ls, sig = [], []
    for r in range(2):
        dn = d[r] / np.linalg.norm(d[r])
        L = chord_length(lo[0], hi[0], o[r], d[r])
        # slab entry over the axes the ray moves along (both rays start inside the z slab)
        t_in = max(min((lo[0][a] - o[r][a]) / dn[a], (hi[0][a] - o[r][a]) / dn[a])
                   for a in range(3) if dn[a] != 0.0)
        Ls.append(L)
        sig.append(fusion.field_sigma(f, o[r] + (t_in + 0.5 * L) * dn))
    assert Ls[0] > 0.02 and Ls[1] > 0.2 and abs(Ls[0] - Ls[1]) > 0.1
    assert abs(v[0, 0] - (Ls[0] * sig[0] + Ls[1] * sig[1]) / (Ls[0] + Ls[1])) < 1e-13
    assert w[0] == pytest.approx(1.0, abs=1e-15)


def test_transmittance_matches_oracle_render(oracle_lib):
    """With tau = 0 the fusion walk ends with the transmittance the oracle
    render reports for the same values as a snapshot (compositing pinned
    elsewhere against closed forms and dense sampling)."""
    dijk = synth.random_tree_leaves(5, 5, p_split=0.6)
    tree = oracle_lib.OracleTree(dijk, 5)
    rng = np.random.default_rng(4)
    vals = np.zeros((len(dijk), 28))
    vals[:, 0] = rng.normal(0.0, 0.3, len(dijk))
    o, d = synth.random_rays(200, 9)
    f = _field()
    _, _, T_end = fusion.observe_rays(oracle_lib, tree, vals, o, d, f, S, 0.0)
    p = oracle_lib.make_params(sigma_scale=S)
    ref = oracle_lib.render_rays(tree, None, p, [0.0], o, d, np.zeros(len(o), np.int32),
                                 snapshot=np.ascontiguousarray(vals.T[None]))
    assert np.allclose(T_end, ref["T"][:, 0], rtol=1e-12, atol=1e-300)
    assert (T_end < 0.999).sum() > 20
