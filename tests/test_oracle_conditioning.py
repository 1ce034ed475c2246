"""Pins for the conditioning helpers that decide which rays are ties of the
colour contract (oracle/conditioning.py), and for the MLP error-scale
helper oracle/mlp.magnitude.

A ray's spread at shift eps is the largest change of its FP64 colour when the
ray moves sideways by eps.  The pins fix it from geometry the helpers do not
use: for a chord between two opposite faces of a box the length does not
depend on a sideways shift (spread 0); for a chord that leaves through a side
face the length changes by eps |w_x / d_x - w_z / d_z| (w the shift
direction), so the colour of one leaf changes by sigma e^(-sigma delta)
|c - bg| times that, to first order (the single-leaf closed form,
C = (1 - e^(-sigma delta)) c + e^(-sigma delta) bg)."""
import math

import numpy as np

from oracle import mlp
from oracle.conditioning import conditioned_reference, perpendicular_pair


def test_perpendicular_pair_orthonormal():
    rng = np.random.default_rng(3)
    d = np.vstack([rng.standard_normal((500, 3)),
                   np.eye(3), -np.eye(3),                     # axis directions (both branches of the helper)
                   [[0.9, 1e-9, 0.0], [1.0, 1e-3, 1e-3], [0.0, 1.0, 1e-12]]])
    u, v = perpendicular_pair(d)
    dn = d / np.linalg.norm(d, axis=1, keepdims=True)
    for a, b in ((u, dn), (v, dn), (u, v)):
        assert np.abs(np.einsum("ij,ij->i", a, b)).max() < 1e-12
    assert np.abs(np.linalg.norm(u, axis=1) - 1).max() < 1e-12
    assert np.abs(np.linalg.norm(v, axis=1) - 1).max() < 1e-12
    # right-handed frame: u x v = d
    assert np.abs(np.cross(u, v) - dn).max() < 1e-12


def _one_leaf(oracle_lib, sigma_raw: float, zdc):
    """Leaf (1, 0, 0, 0) = [0, 0.5]^3 with time-constant density and colour:
    only the DC Fourier terms are set, and only SH j = 0 of each channel."""
    dijk = np.array([[1, 0, 0, 0]], dtype=np.int32)
    k = np.zeros((1, 166))
    k[0, 0] = sigma_raw
    for c in range(3):
        k[0, 31 + (c * 9 + 0) * 5 + 0] = zdc[c]
    return oracle_lib.OracleTree(dijk, 3), k


def test_spread_zero_between_opposite_faces(oracle_lib):
    tree, k = _one_leaf(oracle_lib, 0.05, (0.3, -1.2, 2.0))
    d = np.array([[0.1, 0.2, 1.0]])
    d /= np.linalg.norm(d)
    # through the middle of the leaf: enters z = 0 and leaves z = 0.5 far from every edge
    centre = np.array([0.25, 0.25, 0.25])
    o = centre - 1.3 * d
    p = oracle_lib.make_params(sigma_scale=16.0, bg=(0.1, 0.2, 0.7))
    ref = conditioned_reference(oracle_lib, tree, k, p, [7.0], o, d, np.zeros(1, np.int32), eps=(2e-7, 1e-6))
    assert ref["T"][0, 0] < 0.95                      # the leaf does attenuate the ray
    assert ref["spread"][0] < 1e-12 and ref["spread_wide"][0] < 1e-12


def test_spread_matches_grazing_side_face(oracle_lib):
    sig_raw, s = 0.08, 16.0
    zdc = (0.9, -0.4, 1.7)
    bg = np.array([0.05, 0.6, 0.2])
    tree, k = _one_leaf(oracle_lib, sig_raw, zdc)
    y0 = 0.28209479177387814                          # Y_00
    col = 1.0 / (1.0 + np.exp(-np.array(zdc) * y0))
    sigma = s * sig_raw
    # enters through z = 0 at (0.495, 0.2, 0), leaves through the side face x = 0.5 at a
    # grazing angle (d_x small against d_z)
    entry = np.array([0.495, 0.2, 0.0])
    d = np.array([0.02, 0.01, 1.0])
    d /= np.linalg.norm(d)
    t_exit = (0.5 - entry[0]) / d[0]
    exit_pt = entry + t_exit * d
    assert 0.1 < exit_pt[1] < 0.4 and 0.1 < exit_pt[2] < 0.4   # the exit really is on x = 0.5
    o = entry - 0.7 * d
    delta = t_exit
    p = oracle_lib.make_params(sigma_scale=s, bg=tuple(bg))
    for eps in (2e-7, 1e-6):
        ref = conditioned_reference(oracle_lib, tree, k, p, [3.0], o[None], d[None], np.zeros(1, np.int32),
                                    eps=(eps,))
        c0 = (1 - math.exp(-sigma * delta)) * col + math.exp(-sigma * delta) * bg
        assert np.abs(ref["rgb"][0, 0] - c0).max() < 1e-12
        u, v = perpendicular_pair(d[None])
        dC = sigma * math.exp(-sigma * delta) * np.abs(col - bg)
        want = 0.0
        for w in (u[0], -u[0], v[0], -v[0]):
            d_delta = eps * abs(-w[0] / d[0] + w[2] / d[2])   # exit moves with the side face, entry with z = 0
            want = max(want, float((dC * d_delta).max()))
        got = float(ref["spread"][0])
        assert want > 1e-7
        assert abs(got - want) <= 0.1 * want, (eps, got, want)


def test_magnitude_hand_computed():
    """One path through the network, weights of both signs, a ReLU that is
    off in the real forward pass: the magnitude propagates |terms| and
    ignores the ReLU."""
    w = {"W1": np.zeros((84, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "W3": np.zeros((64, 3)), "b3": np.zeros(3)}
    w["W1"][0, 0] = -2.0        # feature 0 = sin(pi x_0)
    w["b1"][0] = 0.5
    w["W2"][0, 0] = 3.0
    w["b2"][1] = -0.75
    w["W3"][0, 0] = -1.0
    w["W3"][1, 2] = 2.0
    w["b3"][:] = (0.25, -0.5, 0.0)
    x = np.zeros((2, 7))
    x[0, 0] = 0.5               # sin(pi / 2) = 1
    x[1, 0] = 1.0 / 6.0         # sin(pi / 6) = 1/2
    mag = mlp.magnitude(w, x)
    # hidden 0: |g0| 2 + 0.5; layer 2 unit 0: 3 m1_0, unit 1: 0.75; outputs: m2_0 + 0.25, 0.5, 2 * 0.75
    assert np.allclose(mag[0], [2.5 * 3 + 0.25, 0.5, 1.5], rtol=0, atol=1e-12)
    assert np.allclose(mag[1], [1.5 * 3 + 0.25, 0.5, 1.5], rtol=0, atol=1e-12)
    # the real forward pass has hidden unit 0 off (z = -2 + 0.5 < 0): outputs are the biases only
    out, _ = mlp.forward(w, x[:1])
    assert np.allclose(out[0], [0.25, -0.5, 0.0 + 2.0 * 0.0])
    # sign-blind in the weights
    neg = {key: -val for key, val in w.items()}
    assert np.array_equal(mlp.magnitude(neg, x), mag)
