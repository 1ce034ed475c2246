"""The library's ray set-up (fpo_device.h setup_ray_in, host-callable) against
the FP64 slab intersection it computes: clipping a unit-direction ray to an
axis-aligned box (the unit cube, or the leaves' bounds of fpo_leaf_bounds)
gives the entry distance t_in = max(0, max_a min(t1_a, t2_a)) and the chord
t_out - t_in, t_out = min_a max(t1_a, t2_a), with t1_a, t2_a the crossings of
the box's two faces on axis a; a ray hits iff t_in < t_out.  With the unit
cube the result equals setup_ray's bit for bit, and tree_dev turns lattice
bounds into exact cube units.  The driver (tests/native/ray_setup_host.hip) is
built with hipcc; nothing runs on a GPU."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("needs hipcc")
    exe = str(tmp_path_factory.mktemp("ray_setup") / "ray_setup_host")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2202_08614_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "ray_setup_host.hip"), "-o", exe],
                   check=True, capture_output=True, text=True)
    return exe


def _run(exe, rows: np.ndarray):
    text = "\n".join(" ".join(f"{v:.9g}" for v in r) for r in rows.astype(np.float32)) + "\n"
    res = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr[-2000:]
    lines = res.stdout.strip().splitlines()
    out = [ln.split() for ln in lines[1:]]
    return lines[0], out


def _slab(o, d, lo, hi):
    """FP64 definition: entry distance and chord of the unit-direction ray."""
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo - o) / d
        t2 = (hi - o) / d
    par = d == 0
    inside = (o >= lo) & (o <= hi)
    t1 = np.where(par, np.where(inside, -np.inf, np.inf), t1)
    t2 = np.where(par, np.inf, t2)
    t_in = np.maximum(np.minimum(t1, t2).max(1), 0.0)
    t_out = np.maximum(t1, t2).min(1)
    return t_in, t_out, d


def test_tree_dev_bounds_in_cube_units(driver):
    head, _ = _run(driver, np.zeros((0, 12)))
    a, c = head.split("|")
    assert [float(v) for v in a.split()[1:]] == [161 / 512, 174 / 512, 176 / 512, 347 / 512, 349 / 512, 332 / 512]
    assert [float(v) for v in c.split()] == [0, 0, 0, 1, 1, 1]


def test_clip_to_box_matches_slab_definition(driver):
    rng = np.random.default_rng(2202)
    n = 6000
    # boxes on random lattices; rays from a sphere around the cube (some from inside the box)
    D = rng.integers(1, 11, n)
    G = (1 << D).astype(np.float64)
    a = rng.integers(0, G[:, None], (n, 3)).astype(np.float64)
    b = rng.integers(0, G[:, None], (n, 3)).astype(np.float64)
    lo = np.minimum(a, b) / G[:, None]
    hi = (np.maximum(a, b) + 1) / G[:, None]
    u = rng.standard_normal((n, 3))
    o = 0.5 + 1.5 * u / np.linalg.norm(u, axis=1, keepdims=True)
    inner = rng.random(n) < 0.1
    o[inner] = lo[inner] + rng.random((inner.sum(), 3)) * (hi[inner] - lo[inner])
    target = -0.2 + 1.4 * rng.random((n, 3))
    d = target - o
    par = rng.random(n) < 0.1                        # rays parallel to an axis or a face
    d[par, rng.integers(0, 3, par.sum())] = 0.0
    o = o.astype(np.float32).astype(np.float64)
    d = d.astype(np.float32).astype(np.float64)
    unit = rng.random(n) < 0.1                       # the unit cube itself
    lo[unit], hi[unit] = 0.0, 1.0
    rows = np.concatenate([o, d, lo, hi], 1)
    _, out = _run(driver, rows)
    assert len(out) == n
    hit = np.array([int(r[0]) for r in out], bool)
    vals = np.array([[float(x) for x in r[1:6]] for r in out])
    same = np.array([r[6] for r in out])
    t_in, t_out, dn = _slab(o, d, lo, hi)
    clear_hit = t_out - t_in > 1e-5
    clear_miss = t_in - t_out > 1e-5
    assert clear_hit.sum() > n // 4 and clear_miss.sum() > n // 4
    assert hit[clear_hit].all() and not hit[clear_miss].any()
    # FP32 arithmetic at distances up to about 2: a few ulps
    assert np.abs(vals[clear_hit, 0] - t_in[clear_hit]).max() < 2e-6
    assert np.abs(vals[clear_hit, 1] - (t_out - t_in)[clear_hit]).max() < 4e-6
    entry = vals[clear_hit, 2:5]
    assert (entry >= lo[clear_hit] - 2e-6).all() and (entry <= hi[clear_hit] + 2e-6).all()
    assert np.abs(entry - (o[clear_hit] + t_in[clear_hit, None] * dn[clear_hit])).max() < 4e-6
    # the unit cube (drawn, or a depth-1 box that spans it) reproduces setup_ray bit for bit
    cube = (lo == 0.0).all(1) & (hi == 1.0).all(1)
    assert unit.sum() > 100 and (same[cube] == "1").all() and (same[~cube] == "-").all()
