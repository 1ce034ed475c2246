"""Seeded synthetic inputs for the Fourier PlenOctree render and fine-tune path.

This module only *generates inputs*: leaf sets (octree cells given as depth and
integer cell coordinates), Fourier coefficients, camera poses, time points and
ray samples.  It holds none of the method's arithmetic (no basis functions, no
spherical harmonics, no traversal or compositing), so both the FP64 oracle and
the HIP path can consume what it produces without sharing any of the method.

The paper's scenes are private multi-view captures (Sec. 5, experimental
setup); these generators stand in for them with the shapes the paper states:
a 512^3 grid, SH degree 2 (9 components per channel), n1 = 31 density and
n2 = 5 SH Fourier coefficients (Sec. 5, Table 3), and about 60 frames.

Seeds: geometry 2202, coefficients 8614, ray sampling 2022 (numpy PCG64).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Layout of one leaf (Sec. 4.1, Eq. 6): n1 density coefficients, then for each
# RGB channel c and SH index j (j = l*l + l + m) n2 Fourier coefficients.
N_SIGMA = 31
N_SH_FOURIER = 5
SH_DEGREE = 2
N_SH = (SH_DEGREE + 1) ** 2
N_COEFF = N_SIGMA + 3 * N_SH * N_SH_FOURIER  # 166
PERIOD = 60.0          # T, number of frames the Fourier basis spans
SIGMA_SCALE = 64.0     # density per unit-cube length per unit of ReLU(sigma)

GEOMETRY_SEED = 2202
COEFF_SEED = 8614
RAY_SEED = 2022


@dataclasses.dataclass
class Camera:
    """Pinhole camera: eye position, viewing direction, up hint, vertical FOV."""
    eye: Sequence[float]
    fwd: Sequence[float]
    up: Sequence[float]
    fov_y_deg: float
    width: int
    height: int
    time: float


@dataclasses.dataclass
class Scene:
    name: str
    max_depth: int
    leaf_dijk: np.ndarray          # int32 [L][4]: depth, i, j, k
    coeffs: Optional[np.ndarray]   # float32 [L][166], caller (leaf_dijk) order
    cameras: List[Camera]
    stop_T: float = 0.0
    bg: Sequence[float] = (0.0, 0.0, 0.0)

    @property
    def n_leaves(self) -> int:
        return int(self.leaf_dijk.shape[0])


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
def ring_camera(azimuth: float, elevation: float, radius: float, fov_y_deg: float,
                width: int, height: int, time: float,
                target=(0.5, 0.5, 0.5)) -> Camera:
    """Camera on a sphere around `target` (y up), looking at it.

    azimuth and elevation are in radians.  The eye sits at
    target + radius * (cos(el) cos(az), sin(el), cos(el) sin(az)).
    """
    tx, ty, tz = target
    ex = tx + radius * math.cos(elevation) * math.cos(azimuth)
    ey = ty + radius * math.sin(elevation)
    ez = tz + radius * math.cos(elevation) * math.sin(azimuth)
    eye = np.array([ex, ey, ez], dtype=np.float32)
    fwd = (np.array(target, dtype=np.float64) - eye.astype(np.float64))
    fwd = (fwd / np.linalg.norm(fwd)).astype(np.float32)
    return Camera(eye=[float(v) for v in eye], fwd=[float(v) for v in fwd],
                  up=[0.0, 1.0, 0.0], fov_y_deg=float(fov_y_deg),
                  width=int(width), height=int(height), time=float(time))


# --------------------------------------------------------------------------
# leaf sets
# --------------------------------------------------------------------------
def _cell_centres(depth: int) -> np.ndarray:
    g = 1 << depth
    return (np.arange(g, dtype=np.float64) + 0.5) / g


def shell_leaves(depth: int = 6, radius: float = 0.4, half_width: float = 1.25 / 64) -> np.ndarray:
    """Cells whose centre lies within `half_width` of a sphere of `radius` at the cube centre."""
    c = _cell_centres(depth)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
    ii, jj, kk = np.nonzero(np.abs(r - radius) <= half_width)
    d = np.full(ii.shape, depth)
    return np.stack([d, ii, jj, kk], axis=1).astype(np.int32)


@dataclasses.dataclass
class BlobParams:
    A: np.ndarray    # [8][3] motion amplitude
    f: np.ndarray    # [8] temporal frequency (1 or 2 cycles per period)
    phi: np.ndarray  # [8][3] phase
    w: np.ndarray    # [8] Gaussian width
    a: np.ndarray    # [8] Gaussian weight


def blob_params(seed: int = GEOMETRY_SEED, n_gauss: int = 8) -> BlobParams:
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.uniform(0.05, 0.15, size=(n_gauss, 3))
    f = rng.integers(1, 3, size=n_gauss).astype(np.float64)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(n_gauss, 3))
    w = rng.uniform(0.04, 0.08, size=n_gauss)
    a = rng.uniform(0.5, 1.0, size=n_gauss)
    return BlobParams(A=A, f=f, phi=phi, w=w, a=a)


@dataclasses.dataclass
class Field:
    """Analytic radiance field standing in for the generalizable NeRF that the
    fusion stage queries (Sec. 3): density in stored units and a
    view-dependent colour,
        sigma(x)  = sum_g a_g exp(-|x - mu_g|^2 / (2 w_g^2)),
        c_c(x, d) = 1 / (1 + exp(-(u_c . x + v_c . d + b_c))),  c < 3."""
    mu: np.ndarray   # [G][3]
    w: np.ndarray    # [G]
    a: np.ndarray    # [G]
    u: np.ndarray    # [3][3]
    v: np.ndarray    # [3][3]
    b: np.ndarray    # [3]


def fusion_field(t: float = 22.2, seed: int = GEOMETRY_SEED, gain: float = 0.5) -> Field:
    """The moving blob frozen at time t (the static frame being fused), with
    a smooth colour that depends on position and view direction."""
    p = blob_params(seed)
    mu = 0.5 + p.A * np.sin(2.0 * math.pi * p.f[:, None] * t / PERIOD + p.phi)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    u = rng.normal(0.0, 2.0, size=(3, 3))
    v = rng.normal(0.0, 1.0, size=(3, 3))
    b = rng.normal(0.0, 0.5, size=3)
    return Field(mu=mu, w=p.w.copy(), a=gain * p.a, u=u, v=v, b=b)


def blob_max_field(depth: int, params: BlobParams, n_frames: int = 60,
                   period: float = PERIOD) -> np.ndarray:
    """max over frames t = 0..n_frames-1 of the moving-Gaussian density at every cell centre.

    rho(x, t) = sum_g a_g exp(-|x - mu_g(t)|^2 / (2 w_g^2)),
    mu_g(t) = 0.5 + A_g * sin(2 pi f_g t / T + phi_g).
    Each Gaussian is separable, so one frame is a rank-8 sum of outer products.
    """
    import torch  # CPU only; used for the separable outer products
    g = 1 << depth
    c = torch.from_numpy(_cell_centres(depth)).to(torch.float32)
    M = torch.zeros((g, g * g), dtype=torch.float32)
    for t in range(n_frames):
        mu = 0.5 + params.A * np.sin(2.0 * math.pi * params.f[:, None] * t / period + params.phi)
        mu_t = torch.from_numpy(mu).to(torch.float32)                     # [G8][3]
        inv = torch.from_numpy(1.0 / (2.0 * params.w ** 2)).to(torch.float32)
        ex = torch.exp(-((c[:, None] - mu_t[None, :, 0]) ** 2) * inv[None, :])  # [g][8]
        ey = torch.exp(-((c[:, None] - mu_t[None, :, 1]) ** 2) * inv[None, :])
        ez = torch.exp(-((c[:, None] - mu_t[None, :, 2]) ** 2) * inv[None, :])
        ex = ex * torch.from_numpy(params.a).to(torch.float32)[None, :]
        yz = (ey[:, None, :] * ez[None, :, :]).reshape(g * g, -1)          # [g*g][8]
        rho = ex @ yz.T                                                    # [g][g*g]
        torch.maximum(M, rho, out=M)
    return M.reshape(g, g, g).numpy()


def blob_leaves(depth: int, n_target: int, seed: int = GEOMETRY_SEED,
                n_frames: int = 60) -> np.ndarray:
    """Union over frames of the cells where the moving blob exceeds an iso level.

    The iso level is the order statistic that keeps the `n_target` densest
    cells of the max-over-time field, so the union has n_target leaves (up to
    exact ties).
    """
    M = blob_max_field(depth, blob_params(seed), n_frames=n_frames).reshape(-1)
    k = M.size - n_target
    iso = np.partition(M, k)[k]
    idx = np.nonzero(M >= iso)[0]
    g = 1 << depth
    ii, jj, kk = np.unravel_index(idx, (g, g, g))
    d = np.full(ii.shape, depth)
    return np.stack([d, ii, jj, kk], axis=1).astype(np.int32)


def random_tree_leaves(seed: int, max_depth: int, p_split: float = 0.55,
                       p_leaf: float = 0.7, min_split_depth: int = 1) -> np.ndarray:
    """A random mixed-depth leaf set (no two leaves overlap), for small tests.

    Starting from the root, every cell above `max_depth` is split with
    probability p_split (always below `min_split_depth`); an unsplit cell is a
    leaf with probability p_leaf, else empty.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    stack = [(0, 0, 0, 0)]
    while stack:
        d, i, j, k = stack.pop()
        split = d < min_split_depth or (d < max_depth and rng.random() < p_split)
        if split:
            for o in range(8):
                stack.append((d + 1, 2 * i + (o & 1), 2 * j + ((o >> 1) & 1), 2 * k + ((o >> 2) & 1)))
        elif rng.random() < p_leaf:
            out.append((d, i, j, k))
    arr = np.array(out, dtype=np.int32).reshape(-1, 4)
    perm = rng.permutation(arr.shape[0])
    return arr[perm]


# --------------------------------------------------------------------------
# coefficients
# --------------------------------------------------------------------------
def coeff_std(n_sigma: int = N_SIGMA, n_sh_fourier: int = N_SH_FOURIER) -> np.ndarray:
    """Per-coefficient standard deviation 1/(i+1), i = Fourier index, leaf order."""
    s = [1.0 / (i + 1) for i in range(n_sigma)]
    for _c in range(3):
        for _j in range(N_SH):
            s.extend(1.0 / (i + 1) for i in range(n_sh_fourier))
    return np.array(s, dtype=np.float64)


def gaussian_coeffs(n_leaves: int, seed: int = COEFF_SEED, n_sigma: int = N_SIGMA,
                    n_sh_fourier: int = N_SH_FOURIER, chunk: int = 1 << 18) -> np.ndarray:
    """k_i ~ N(0, 1/(i+1)^2) for every coefficient, float32 [L][n_coeff]."""
    std = coeff_std(n_sigma, n_sh_fourier).astype(np.float32)
    nc = std.size
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n_leaves, nc), dtype=np.float32)
    for s in range(0, n_leaves, chunk):
        e = min(n_leaves, s + chunk)
        out[s:e] = rng.standard_normal((e - s, nc), dtype=np.float32) * std[None, :]
    return out


def perturb_coeffs(coeffs: np.ndarray, sd: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal(coeffs.shape, dtype=np.float32) * np.float32(sd)
    return (coeffs + noise).astype(np.float32)


# --------------------------------------------------------------------------
# the five workload configurations
# --------------------------------------------------------------------------
def c1_scene() -> Scene:
    """Depth-6 spherical shell (radius 0.4, 20,536 leaves), one 64x64 view at t = 0.37 T."""
    dijk = shell_leaves(6, 0.4, 1.25 / 64)
    coeffs = gaussian_coeffs(dijk.shape[0])
    cam = ring_camera(math.radians(30.0), math.radians(20.0), 1.5, 45.0, 64, 64, 0.37 * PERIOD)
    return Scene("c1_shell_d6_64x64", 6, dijk, coeffs, [cam], stop_T=0.0)


def c2_times() -> List[float]:
    return [(j + 0.37) * 6.0 for j in range(10)]


def c2_cameras(width: int = 1920, height: int = 1080, times: Optional[Sequence[float]] = None) -> List[Camera]:
    """16 ring cameras (elevation 15 deg, radius 1.5, FOV 30 deg) x the time points."""
    times = c2_times() if times is None else times
    cams = []
    for t in times:
        for k in range(16):
            cams.append(ring_camera(2.0 * math.pi * k / 16, math.radians(15.0), 1.5, 30.0,
                                    width, height, t))
    return cams


def c2_scene(with_coeffs: bool = True, n_leaves: int = 2_000_000) -> Scene:
    """Depth-9 union of 60 frames of a moving 8-Gaussian blob, 2.0 M leaves."""
    dijk = blob_leaves(9, n_leaves)
    coeffs = gaussian_coeffs(dijk.shape[0]) if with_coeffs else None
    return Scene("c2_blob_d9_2M", 9, dijk, coeffs, c2_cameras(), stop_T=1e-3)


def c3_cameras(width: int = 800, height: int = 800, n: int = 64) -> List[Camera]:
    return [ring_camera(2.0 * math.pi * k / n, math.radians(15.0), 1.5, 30.0, width, height,
                        k * PERIOD / n) for k in range(n)]


def c4_cameras(width: int = 800, height: int = 800) -> List[Camera]:
    """24 ring cameras x 30 times t = (j + 0.5) * 2."""
    cams = []
    for j in range(30):
        t = (j + 0.5) * 2.0
        for k in range(24):
            cams.append(ring_camera(2.0 * math.pi * k / 24, math.radians(15.0), 1.5, 30.0,
                                    width, height, t))
    return cams


def fusion_cameras(n: int = 100, width: int = 800, height: int = 800) -> List[Camera]:
    """Dense views for the fusion stage: azimuths on the golden angle,
    elevations spread over [-40, 40] degrees, radius 1.6, FOV 40 degrees."""
    golden = (math.sqrt(5.0) - 1.0) / 2.0
    return [ring_camera(2.0 * math.pi * ((k * golden) % 1.0), math.radians(-40.0 + 80.0 * (k + 0.5) / n), 1.6,
                        40.0, width, height, 0.0) for k in range(n)]


def c4_scene(n_leaves: int = 500_000) -> Scene:
    dijk = blob_leaves(8, n_leaves)
    coeffs = gaussian_coeffs(dijk.shape[0])
    return Scene("c4_blob_d8_500k", 8, dijk, coeffs, c4_cameras(), stop_T=1e-3)


def blob_peak_frames(leaf_dijk: np.ndarray, params: BlobParams, n_frames: int = 60,
                     period: float = PERIOD, chunk: int = 1 << 19) -> np.ndarray:
    """For every leaf, the frame (0..n_frames-1) at which the moving blob's
    density rho(x, t) at the leaf's centre is largest."""
    import torch  # CPU only
    d = leaf_dijk[:, 0].astype(np.float64)
    centre = (leaf_dijk[:, 1:4].astype(np.float64) + 0.5) / (2.0 ** d)[:, None]
    inv = torch.from_numpy(1.0 / (2.0 * params.w ** 2))
    a = torch.from_numpy(params.a)
    out = np.empty(len(leaf_dijk), np.int32)
    mus = [torch.from_numpy(0.5 + params.A * np.sin(2.0 * math.pi * params.f[:, None] * t / period + params.phi))
           for t in range(n_frames)]
    for s in range(0, len(leaf_dijk), chunk):
        x = torch.from_numpy(centre[s:s + chunk])                              # [n][3]
        best = torch.full((x.shape[0],), -1.0, dtype=torch.float64)
        arg = torch.zeros((x.shape[0],), dtype=torch.int32)
        for t, mu in enumerate(mus):
            r2 = ((x[:, None, :] - mu[None, :, :]) ** 2).sum(-1)                # [n][8]
            rho = (a[None, :] * torch.exp(-r2 * inv[None, :])).sum(-1)
            better = rho > best
            best = torch.where(better, rho, best)
            arg = torch.where(better, torch.full_like(arg, t), arg)
        out[s:s + chunk] = arg.numpy()
    return out


def pulse_coeffs(leaf_dijk: np.ndarray, seed: int = COEFF_SEED, geometry_seed: int = GEOMETRY_SEED,
                 n_frames: int = 60, width: float = 3.0, threshold: float = 0.5) -> np.ndarray:
    """Coefficients whose density follows the moving blob in time: each
    leaf's density is a periodic pulse centred on its peak frame tau (the frame
    at which the blob is densest there), negative elsewhere,
        sigma(t) = A (P(t - tau) - threshold),
        P(u) = sum_{m <= 15} g_m cos(2 pi m u / T) / sum_m g_m,  g_m = exp(-m^2 / (2 width^2)),
    with A ~ U[1, 3] per leaf, so that a leaf is dense for a few frames around
    tau and transparent (sigma <= 0) the rest of the period, as a region of a
    moving object is.  In the coefficient order of Eq. 8 a harmonic m is the
    pair (sin, cos) at indices (2m - 1, 2m): k_{2m-1} = A g_m sin(2 pi m tau / T)
    / Z, k_{2m} = A g_m cos(2 pi m tau / T) / Z.  The SH colour coefficients are
    N(0, 1/(i+1)^2) as elsewhere."""
    tau = blob_peak_frames(leaf_dijk, blob_params(geometry_seed), n_frames=n_frames).astype(np.float64)
    k = gaussian_coeffs(len(leaf_dijk), seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 101))
    amp = rng.uniform(1.0, 3.0, size=len(leaf_dijk))
    n_harm = (N_SIGMA - 1) // 2
    g = np.exp(-np.arange(n_harm + 1) ** 2 / (2.0 * width ** 2))
    Z = g.sum()
    k[:, 0] = (amp * (g[0] / Z - threshold)).astype(np.float32)
    for m in range(1, n_harm + 1):
        ph = 2.0 * math.pi * m * tau / PERIOD
        k[:, 2 * m - 1] = (amp * g[m] / Z * np.sin(ph)).astype(np.float32)
        k[:, 2 * m] = (amp * g[m] / Z * np.cos(ph)).astype(np.float32)
    return k


def c5_pulse_scene() -> Scene:
    """The depth-9 blob union (2.0 M leaves, as in the headline scene) with
    pulse densities (pulse_coeffs): at any time only the part of the union the
    blob occupies then is dense, the rest of its trail is transparent."""
    dijk = blob_leaves(9, 2_000_000)
    return Scene("c5_blob_d9_pulse", 9, dijk, pulse_coeffs(dijk), c5_test_cameras(), stop_T=1e-3)


def sample_pixels(n: int, n_cams: int, width: int, height: int, seed: int = RAY_SEED):
    """Uniform (camera, row, column) triples."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cam = rng.integers(0, n_cams, size=n)
    py = rng.integers(0, height, size=n)
    px = rng.integers(0, width, size=n)
    return cam.astype(np.int32), py.astype(np.int32), px.astype(np.int32)


def random_rays(n: int, seed: int, inside_frac: float = 0.2):
    """Random rays aimed at the unit cube, float32 origins/directions.

    Most origins lie on a sphere of radius 1.5 around the cube centre and aim
    at a random point of the cube; a fraction start inside the cube.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    o = 0.5 + 1.5 * v
    target = rng.uniform(0.0, 1.0, size=(n, 3))
    inside = rng.random(n) < inside_frac
    o[inside] = rng.uniform(0.05, 0.95, size=(int(inside.sum()), 3))
    d = target - o
    d[inside] = rng.standard_normal((int(inside.sum()), 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


# --------------------------------------------------------------------------
# learned-proposal workload: depth-9 blob scene, training rays from random ring
# cameras, test views = the 16 ring cameras x 30 times
# --------------------------------------------------------------------------
C5_N_TIMES = 3600     # training times: a grid of T / 3600 over the period


def c5_time_grid() -> np.ndarray:
    return (np.arange(C5_N_TIMES) + 0.5) * (PERIOD / C5_N_TIMES)


def c5_train_cameras(n_cams: int = 4096, width: int = 1920, height: int = 1080,
                     seed: int = RAY_SEED) -> List[Camera]:
    """Ring cameras at azimuth U[0, 2 pi), elevation U[5, 25] deg, radius 1.5,
    FOV 30 deg (their time is unused: each training ray draws its own)."""
    rng = np.random.Generator(np.random.PCG64(seed + 5))
    az = rng.uniform(0.0, 2.0 * math.pi, n_cams)
    el = np.radians(rng.uniform(5.0, 25.0, n_cams))
    return [ring_camera(float(a), float(e), 1.5, 30.0, width, height, 0.0) for a, e in zip(az, el)]


def c5_train_samples(n: int, n_cams: int, width: int = 1920, height: int = 1080, seed: int = RAY_SEED):
    """(camera, row, column, time index) of n training rays, uniform."""
    rng = np.random.Generator(np.random.PCG64(seed + 6))
    cam = rng.integers(0, n_cams, size=n).astype(np.int32)
    py = rng.integers(0, height, size=n).astype(np.int32)
    px = rng.integers(0, width, size=n).astype(np.int32)
    t_idx = rng.integers(0, C5_N_TIMES, size=n).astype(np.int32)
    return cam, py, px, t_idx


def c5_test_cameras(width: int = 1920, height: int = 1080) -> List[Camera]:
    """The 16 C2 ring cameras at 30 times t = (j + 0.5) * 2."""
    return c2_cameras(width, height, times=[(j + 0.5) * 2.0 for j in range(30)])


def mlp_init(seed: int = 11) -> np.ndarray:
    """He-normal proposal weights with zero biases, as the flat FP32 vector
    ([85][64], [65][64], [65][3], bias rows last), padded to 9796."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for n_in, n_out in ((84, 64), (64, 64), (64, 3)):
        w = rng.standard_normal((n_in, n_out)) * math.sqrt(2.0 / n_in)
        parts.append(np.vstack([w, np.zeros((1, n_out))]).ravel())
    p = np.zeros(9796, np.float32)
    flat = np.concatenate(parts)
    p[:flat.size] = flat
    return p


# --------------------------------------------------------------------------
# per-frame PlenOctrees (inputs of the FPO construction): the blob sampled at
# every frame, standing in for the per-frame fusion results
# --------------------------------------------------------------------------
def blob_frame_leaves(depth: int, n_union: int, n_frames: int = 60, seed: int = GEOMETRY_SEED,
                      merge_every: int = 4) -> List[np.ndarray]:
    """Frame t holds the cells of the union iso set (`blob_leaves`) whose
    density at t exceeds the same iso level; where all eight children of a
    parent are present, frame t keeps the parent instead for one in
    `merge_every` (parent, frame) pairs, so frames differ in depth and the
    union splits their coarser leaves."""
    params = blob_params(seed)
    M = blob_max_field(depth, params, n_frames=n_frames).reshape(-1)
    k = M.size - n_union
    iso = np.partition(M, k)[k]
    cells = blob_leaves(depth, n_union, seed, n_frames)
    import torch  # CPU only, as in blob_max_field
    g = 1 << depth
    x = torch.from_numpy((cells[:, 1:4].astype(np.float32) + 0.5) / g)
    inv_w = torch.from_numpy((1.0 / (2.0 * params.w ** 2)).astype(np.float32))
    amp = torch.from_numpy(params.a.astype(np.float32))
    out = []
    for t in range(n_frames):
        mu = 0.5 + params.A * np.sin(2.0 * math.pi * params.f[:, None] * t / PERIOD + params.phi)
        mu_t = torch.from_numpy(mu.astype(np.float32))                      # [G][3]
        r2 = ((x[:, None, :] - mu_t[None]) ** 2).sum(-1)                    # [n][G]
        rho = (torch.exp(-r2 * inv_w[None]) * amp[None]).sum(-1).numpy()
        sel = cells[rho >= iso]
        par = sel[:, 1:4] >> 1
        key = (par[:, 0].astype(np.int64) * g + par[:, 1]) * g + par[:, 2]
        uk, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
        h = (uk * 2654435761 + t * 40503) % merge_every
        full = (cnt[inv] == 8) & (h[inv] == 0)
        keep = sel[~full]
        pk = np.unique(key[full])
        pi = np.stack([np.full(len(pk), depth - 1), pk // (g * g), (pk // g) % g, pk % g], axis=1)
        out.append(np.concatenate([keep, pi.astype(np.int32)]).astype(np.int32))
    return out
