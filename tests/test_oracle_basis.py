"""Pins for the oracle's real Fourier basis (Eq. 8) and spherical harmonics (Eq. 1)."""
import math

import numpy as np
import pytest

T = 60.0


def test_basis_closed_values(oracle_lib):
    b = oracle_lib.basis(0.0, T, 31)
    # at t = 0: cos terms are 1, sin terms 0
    assert np.allclose(b[0::2], 1.0, atol=0) and np.allclose(b[1::2], 0.0, atol=1e-15)
    # b_1(T/4) = sin(2 pi / 4) = 1, b_2(T/4) = cos(pi/2) = 0
    b = oracle_lib.basis(T / 4, T, 31)
    assert b[0] == 1.0
    assert abs(b[1] - 1.0) < 1e-15 and abs(b[2]) < 1e-15
    # t = T/2: even i -> (-1)^(i/2), odd i -> sin(k pi) = 0
    b = oracle_lib.basis(T / 2, T, 31)
    assert np.allclose(b[0::2], [(-1) ** (i // 2) for i in range(0, 31, 2)], atol=1e-14)
    assert np.allclose(b[1::2], 0.0, atol=1e-13)


def test_basis_periodic(oracle_lib):
    rng = np.random.default_rng(1)
    for t in rng.uniform(-100, 100, size=20):
        assert np.allclose(oracle_lib.basis(t, T, 31), oracle_lib.basis(t + T, T, 31), atol=1e-12)


def test_basis_orthogonal_on_frames(oracle_lib):
    """sum_{t=0}^{T-1} b_i b_j = T [i=j=0] + T/2 [i=j>=1] (frequencies stay below T/2)."""
    B = np.stack([oracle_lib.basis(t, T, 31) for t in range(int(T))])
    G = B.T @ B
    expect = np.diag([T] + [T / 2] * 30)
    assert np.max(np.abs(G - expect)) < 1e-11


def test_basis_matches_fft_bins(oracle_lib):
    """Index pin against numpy's FFT: b_i over t = 0..T-1 has exactly one
    spectral line, at k = ceil(i/2) cycles per period; even i is a cosine
    (real bin +T/2, or T for i = 0), odd i a sine (imaginary bin -T/2)."""
    n = int(T)
    B = np.stack([oracle_lib.basis(t, T, 31) for t in range(n)])
    for i in range(31):
        X = np.fft.rfft(B[:, i])
        k = (i + 1) // 2
        expect = np.zeros_like(X)
        if i == 0:
            expect[0] = n
        elif i % 2 == 0:
            expect[k] = n / 2
        else:
            expect[k] = -1j * n / 2
        assert np.max(np.abs(X - expect)) < 1e-10, i


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def test_sh_constant_and_scipy(oracle_lib):
    from oracle.brute import real_sh9_scipy
    assert abs(oracle_lib.sh9([0, 0, 1])[0] - 1.0 / (2.0 * math.sqrt(math.pi))) < 1e-15
    rng = np.random.default_rng(2)
    for _ in range(50):
        d = _unit(rng.standard_normal(3))
        assert np.allclose(oracle_lib.sh9(d), real_sh9_scipy(d), atol=1e-13)


def test_sh_orthonormal_quadrature(oracle_lib):
    """int Y_a Y_b dOmega = delta_ab by Gauss-Legendre in cos(theta) x uniform phi."""
    nx, nphi = 16, 32
    x, w = np.polynomial.legendre.leggauss(nx)
    G = np.zeros((9, 9))
    for xi, wi in zip(x, w):
        s = math.sqrt(1 - xi * xi)
        for k in range(nphi):
            phi = 2 * math.pi * k / nphi
            Y = oracle_lib.sh9([s * math.cos(phi), s * math.sin(phi), xi])
            G += wi * (2 * math.pi / nphi) * np.outer(Y, Y)
    assert np.max(np.abs(G - np.eye(9))) < 1e-12


def test_sh_addition_theorem(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(20):
        Y = oracle_lib.sh9(_unit(rng.standard_normal(3)))
        for l in range(3):
            s = sum(Y[l * l + l + m] ** 2 for m in range(-l, l + 1))
            assert abs(s - (2 * l + 1) / (4 * math.pi)) < 1e-13


@pytest.mark.parametrize("W,H", [(3, 3), (5, 7)])
def test_camera_geometry(oracle_lib, W, H):
    from paper_2202_08614_amd.synth import Camera
    cam = Camera(eye=[0.5, 0.5, 2.0], fwd=[0, 0, -1], up=[0, 1, 0], fov_y_deg=40.0,
                 width=W, height=H, time=0.0)
    # centre pixel looks straight ahead
    o, d = oracle_lib.camera_rays(cam, np.array([W // 2]), np.array([H // 2]))
    assert np.allclose(o[0], cam.eye) and np.allclose(d[0], [0, 0, -1], atol=1e-15)
    # top row is above the centre (y up), first column on the left (-x for this pose)
    o, d = oracle_lib.camera_rays(cam, np.array([0]), np.array([0]))
    tan_h = math.tan(math.radians(20.0))
    sy = (1 - 1.0 / H) * tan_h
    sx = -(1 - 1.0 / W) * tan_h * W / H
    expect = _unit([sx, sy, -1.0])
    assert np.allclose(d[0], expect, atol=1e-15)
