"""Pins for opacity acceleration (section "Transparency rendering": with a
LoD, step size and sampled level grow with the optical depth, after Danskin
and Hanrahan) and its colour pyramid.

Reading: once the accumulated optical depth -ln(1 - A) reaches accel_depth,
the ray leaves the lines at the end of the current voxel and samples the
density pyramid: level l = min(top, 1 + floor(log2(delta / accel_depth))),
step D = 2^l, sample at the step's midpoint, opacity min(1, rho D), colour
the density-weighted mean colour rgb / rho, front-to-back until alpha_stop or
the grid's edge. Contract: the image differs from the exact one by at most
e^-accel_depth per channel (the transmittance left at the switch).

Each pin fails under a plausible slip: the colour pyramid's sigma or length
weight dropped, the switch taken before the threshold or never, samples
taken at the step's start instead of its midpoint, the level not rising
with the depth, or the colour not divided by the density."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1801_01155_amd import synth


def _code(face, bu, bw):
    return face | (bu << 3) | (bw << 9)


def _rec(entry, exit_, attr=255, curve=0):
    return entry | (exit_ << 15) | (attr << 32) | (curve << 40)


def _stack(grid, n, z0):
    """n straight lines along x through the row y = 8 at z = z0, z0 + 1, ...
    (bins 16 of 32: y = z = 8 + 33/64 local), each its own curve, attribute 200."""
    G = grid
    lists = {}
    for k in range(n):
        for x in range(G[0]):
            v = x + G[0] * (8 + G[1] * (z0 + k))
            lists.setdefault(v, []).append(_rec(_code(0, 16, 16), _code(1, 16, 16), 200, k))
    nvox = int(np.prod(G))
    offs, recs = [0], []
    for v in range(nvox):
        recs += lists.get(v, [])
        offs.append(len(recs))
    return O.OracleCsr(np.array(offs, np.uint32), np.array(recs, np.uint64), 0, 0)


def _down_cam(x, y, z):
    return synth.Camera((x, y, z), (0.0, 0.0, -1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 1, 1, True)


# --- colour pyramid -----------------------------------------------------------------------
def test_color_pyramid_single_line_and_mass_conservation():
    rng = np.random.default_rng(3)
    grid = (12, 10, 9)
    verts, off = [], [0]
    for _ in range(30):
        p = rng.integers(256, np.array(grid) * 256 - 256)
        pts = [p]
        for _ in range(6):
            pts.append(np.clip(pts[-1] + rng.integers(-400, 401, 3), 0, np.array(grid) * 256 - 1))
        verts += pts
        off.append(len(verts))
    attr = rng.integers(0, 256, 30).astype(np.uint8)
    csr = O.voxelize(np.array(verts, np.int32), np.array(off, np.int64), attr, grid, 16)
    lut = synth.lut_importance_alpha()
    rgb = O.lod_color(csr, grid, 16, lut, opaque=False)
    _, _, rho, dims, loff = O.lod(csr, grid, 16, lut, opaque=False)
    # level 0 by hand: sum of length * sigma * colour
    want = np.zeros((int(loff[1]), 3))
    for v in range(int(loff[1])):
        for r in csr.records[csr.offsets[v]:csr.offsets[v + 1]]:
            a, b = O.decode(int(r), 16)
            at = (int(r) >> 32) & 0xFF
            want[v] += np.linalg.norm(b - a) * float(lut[at, 3]) * lut[at, :3].astype(np.float64)
    assert np.allclose(rgb[:loff[1]], want, rtol=1e-12, atol=1e-12)
    for lv in range(len(dims)):
        s = rgb[loff[lv]:loff[lv + 1]].sum(axis=0) * 8.0 ** lv
        assert np.allclose(s, want.sum(axis=0), rtol=1e-10)
    # the mean colour of a cell lies inside the transfer function's colour range
    m = rho > 0
    mean = rgb[m] / rho[m, None]
    lut64 = lut.astype(np.float64)
    assert (mean >= lut64[:, :3].min(axis=0) - 1e-9).all()
    assert (mean <= lut64[:, :3].max(axis=0) + 1e-9).all()


# --- switch rule, truncation, contract ----------------------------------------------------
def _pyr(grid, rho_levels=None, rgb_levels=None):
    dims, loff = O.lod_levels(grid)
    rho = np.zeros(int(loff[-1]))
    rgb = np.zeros((int(loff[-1]), 3))
    for lv in range(len(dims)):
        if rho_levels is not None:
            rho[loff[lv]:loff[lv + 1]] = rho_levels(lv)
        if rgb_levels is not None:
            rgb[loff[lv]:loff[lv + 1]] = rgb_levels(lv)
    return rho, rgb, dims, loff


@pytest.mark.parametrize("depth0", [0.3, 0.9, 2.0])
def test_switch_truncates_at_the_threshold_over_empty_density(depth0):
    """Lines of alpha a stacked below the camera, an empty pyramid: the
    accelerated image is the exact one cut after the first fragment that
    brings -ln(1 - A) to depth0: A = 1 - (1 - a)^k*, k* = ceil(depth0 / -ln(1 - a))."""
    grid = (16, 16, 16)
    csr = _stack(grid, 10, 2)
    a = float(np.float32(0.3))      # the transfer function stores fp32
    lut = synth.lut_constant((0.2, 0.6, 0.9), a)
    rho, rgb, _, _ = _pyr(grid)
    cam = _down_cam(5.5, 8 + 33 / 64, 40.0)
    kw = dict(lut=lut, radius=0.4, opaque=False, shading=0, mode=0, alpha_stop=0.99,
              merge_curves=True)
    exact, _ = O.render(csr, grid, 32, cam, **kw)
    acc, _ = O.render(csr, grid, 32, cam, rho=rho, rgb=rgb, accel_depth=depth0, **kw)
    kstar = math.ceil(depth0 / -math.log(1 - a) - 1e-12)
    A = 1 - (1 - a) ** kstar
    assert acc[0, 0, 3] == pytest.approx(A, abs=1e-12)
    assert np.allclose(acc[0, 0, :3], np.array([0.2, 0.6, 0.9], np.float32) * A, atol=1e-9)
    assert exact[0, 0, 3] == pytest.approx(1 - (1 - a) ** 10, abs=1e-12)
    # off: identical to the exact render
    off, _ = O.render(csr, grid, 32, cam, rho=rho, rgb=rgb, accel_depth=0.0, **kw)
    assert np.array_equal(off, exact)


def _uniform_medium(A_sw, z_switch, depth0, rho0, c0, top, alpha_stop):
    """Density steps of the reading in a uniform medium (rho0, colour c0 on
    every level) from the switch point down to z = 0."""
    C = np.zeros(3)
    A = A_sw
    s = 0.0
    while A < alpha_stop:
        lv = min(top, 1 + int(math.floor(math.log2(-math.log(1 - A) / depth0))))
        D = 2.0 ** lv
        if not (z_switch - (s + D / 2) >= 0):
            break
        al = min(1.0, rho0 * D)
        C += (1 - A) * al * c0
        A += (1 - A) * al
        s += D
    return C, A


@pytest.mark.parametrize("rho0", [0.01, 0.05, 1.0])
def test_uniform_medium_after_the_switch(rho0):
    """One line at z ~ 14.5 (alpha 0.6 > 1 - e^-0.5) switches in voxel
    z = 14; below it a uniform medium: steps of 2, 4, 8 ... voxels as the
    optical depth doubles, each min(1, rho0 D) of colour c0."""
    grid = (16, 16, 16)
    csr = _stack(grid, 1, 14)
    a = float(np.float32(0.6))
    cl = np.array([0.9, 0.1, 0.1])
    lut = synth.lut_constant(tuple(cl), a)
    c0 = np.array([0.1, 0.4, 0.7])
    rho, rgb, dims, _ = _pyr(grid, lambda lv: rho0, lambda lv: rho0 * c0)
    cam = _down_cam(5.5, 8 + 33 / 64, 40.0)
    depth0 = 0.5
    img, _ = O.render(csr, grid, 32, cam, lut=lut, radius=0.4, opaque=False, shading=0, mode=0,
                      alpha_stop=0.999, rho=rho, rgb=rgb, accel_depth=depth0)
    C_m, A = _uniform_medium(a, 14.0, depth0, rho0, c0, len(dims) - 1, 0.999)
    C = cl.astype(np.float32).astype(np.float64) * a + C_m
    assert img[0, 0, 3] == pytest.approx(A, abs=1e-9)
    assert np.allclose(img[0, 0, :3], C, atol=1e-9)
    if rho0 == 1.0:
        # one saturating step: all the remaining light takes the medium's colour
        assert img[0, 0, 3] == 1.0
        assert np.allclose(img[0, 0, :3], cl.astype(np.float32) * a + (1 - a) * c0, atol=1e-9)


def test_level_rises_with_depth():
    """Distinct colours per level: the first step after the switch (depth in
    [depth0, 2 depth0)) samples level 1; later steps coarser levels."""
    grid = (64, 16, 16)
    csr = _stack(grid, 1, 14)
    a = 0.5
    lut = synth.lut_constant((0.0, 0.0, 0.0), a)   # 0.5 is exact in fp32
    cols = {1: np.array([1.0, 0, 0]), 2: np.array([0, 1.0, 0]), 3: np.array([0, 0, 1.0])}
    rho0 = 0.15
    rho, rgb, dims, _ = _pyr(grid, lambda lv: rho0,
                             lambda lv: rho0 * cols.get(lv, np.array([0.5, 0.5, 0.5])))
    cam = _down_cam(5.5, 8 + 33 / 64, 40.0)
    depth0 = -math.log(1 - a)       # the switch happens right at the first line
    img, _ = O.render(csr, grid, 32, cam, lut=lut, radius=0.4, opaque=False, shading=0, mode=0,
                      alpha_stop=0.999, rho=rho, rgb=rgb, accel_depth=depth0 * 0.999)
    # steps: level 1 (D = 2) while delta < 2 depth0, then level 2 (D = 4), ...
    C = np.zeros(3)
    A, s = a, 0.0
    while True:
        lv = min(len(dims) - 1, 1 + int(math.floor(math.log2(-math.log(1 - A) / (depth0 * 0.999)))))
        D = 2.0 ** lv
        if 14.0 - (s + D / 2) < 0:
            break
        al = min(1.0, rho0 * D)
        C += (1 - A) * al * cols.get(lv, np.array([0.5, 0.5, 0.5]))
        A += (1 - A) * al
        s += D
    assert np.allclose(img[0, 0, :3], C, atol=1e-9)
    assert img[0, 0, 0] > 0 and img[0, 0, 1] > 0      # levels 1 and 2 both sampled


@pytest.mark.parametrize("depth0", [0.5, 1.2])
def test_error_contract_on_streamlines(depth0):
    """|accelerated - exact| <= e^-depth0 per channel on every pixel."""
    ls = synth.abc_lineset(600, 120, 17, perturb=True)
    grid = 48
    lat, _, _ = O.grid_setup(ls.xyz, grid)
    csr = O.voxelize(lat, ls.curve_off, ls.attr, grid, 32)
    lut = synth.lut_importance_alpha(0.1, 0.7)
    _, _, rho, _, _ = O.lod(csr, grid, 32, lut, opaque=False)
    rgb = O.lod_color(csr, grid, 32, lut, opaque=False)
    cam = synth.default_camera((grid,) * 3, 48, 32)
    kw = dict(lut=lut, radius=0.4, opaque=False, shading=1, alpha_stop=0.99)
    exact, _ = O.render(csr, grid, 32, cam, **kw)
    acc, _ = O.render(csr, grid, 32, cam, rho=rho, rgb=rgb, accel_depth=depth0, **kw)
    bound = math.exp(-depth0)
    err = np.abs(acc - exact).max()
    print(f"accel depth0={depth0}: max |acc - exact| = {err:.4f} <= {bound:.4f}")
    assert err <= bound + 1e-12
    assert np.abs(acc - exact).max() > 1e-4     # it does change the image
