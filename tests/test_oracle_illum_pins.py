"""Pins for the oracle's cone directions, occlusion grids and AO/shadow shading.

Sections "Shadow simulation" (one cone towards the light, density sampled
along it), "Ambient occlusion" (cones over the whole sphere around a voxel,
occlusion accumulated up to 1, averaged over the cones) and "Rendering
effects" (local illumination at the tube entry point). Each pin is chosen
so that a plausible slip fails it: a wrong golden angle or z spacing in the
spherical Fibonacci set, a shadow cone traced away from the light, AO
reported as occlusion instead of 1 - occlusion, the AO factor dropped from
the ambient term, the light direction flipped, the half vector replaced by
the view vector, or the grids looked up at the voxel centre instead of the
entry point.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1801_01155_amd import synth


# --- spherical Fibonacci directions ---------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 5, 16, 32])
def test_fibonacci_dirs_definition(n):
    d = O.fibonacci_dirs(n)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    # heights equally spaced by 2/n, from 1 - 1/n down to -1 + 1/n
    z = d[:, 2]
    assert math.isclose(z[0], 1.0 - 1.0 / n, abs_tol=1e-15)
    assert np.allclose(np.diff(z), -2.0 / n, atol=1e-14)
    assert math.isclose(z[-1], -1.0 + 1.0 / n, abs_tol=1e-14)
    # consecutive azimuths differ by the golden angle 2 pi / phi^2 (mod 2 pi)
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    golden = 2.0 * math.pi / (phi * phi)
    az = np.arctan2(d[:, 1], d[:, 0])
    ok = np.hypot(d[:, 0], d[:, 1]) > 1e-9
    for i in range(n - 1):
        if ok[i] and ok[i + 1]:
            step = (az[i + 1] - az[i]) % (2.0 * math.pi)
            assert math.isclose(step, golden, abs_tol=1e-12)
    # the first direction sits at azimuth 0
    if ok[0]:
        assert abs(az[0]) < 1e-15


def test_fibonacci_dirs_balanced():
    # the set is symmetric in z and spreads azimuth: its mean tends to 0
    d = O.fibonacci_dirs(256)
    assert abs(d[:, 2].sum()) < 1e-12
    assert np.abs(d.mean(axis=0)).max() < 0.02


# --- AO grid: saturating half-space ---------------------------------------------------
def _level0_pyramid(grid, level0):
    dims, loff = O.lod_levels(grid)
    rho = np.zeros(int(loff[-1]))
    rho[:loff[1]] = level0.ravel()
    return rho


@pytest.mark.parametrize("n", [16, 7])
def test_ao_dense_half_space_below(n):
    """A saturating half-space z < 16 below the voxel at z = 16: every cone
    heading down (d_z < 0) is fully blocked at its first unit step, every
    other cone sees nothing (aperture 0 keeps all samples on level 0 at unit
    steps). AO = 1 - (number of cones with d_z < 0) / n: 8/16 blocked for
    n = 16; for n = 7 one cone is exactly horizontal and stays clear, so 3/7
    are blocked."""
    g = (32, 32, 32)
    lvl0 = np.zeros((32, 32, 32))                 # [z, y, x]
    lvl0[:16] = 1e3
    rho = _level0_pyramid(g, lvl0)
    ao = O.ao_grid(rho, g, n_cones=n, radius=15.0, aperture=0.0).reshape(32, 32, 32)
    down = int((O.fibonacci_dirs(n)[:, 2] < 0).sum())
    assert down == (8 if n == 16 else 3)
    assert math.isclose(ao[16, 16, 16], 1.0 - down / n, abs_tol=1e-12)
    # inside the dense half every cone saturates at once: AO = 0
    assert ao[4, 16, 16] == 0.0
    # a cone straight up from just above the boundary is clear, straight down is blocked
    p = np.array([16.5, 16.5, 16.5])
    assert O.cone(rho, g, p, [0, 0, 1], 15.0, aperture=0.0) == 0.0
    assert O.cone(rho, g, p, [0, 0, -1], 15.0, aperture=0.0) == 1.0


def test_ao_half_space_along_x_depends_on_azimuth():
    """The same saturating half-space, now x < 16: the blocked cones are
    those with d_x < 0, which depends on the azimuths of the set."""
    g = (32, 32, 32)
    lvl0 = np.zeros((32, 32, 32))
    lvl0[:, :, :16] = 1e3
    rho = _level0_pyramid(g, lvl0)
    ao = O.ao_grid(rho, g, n_cones=16, radius=15.0, aperture=0.0).reshape(32, 32, 32)
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    k = np.arange(16)
    zk = 1.0 - (2.0 * k + 1.0) / 16.0
    xk = np.sqrt(1.0 - zk * zk) * np.cos(2.0 * math.pi * k / (phi * phi))
    blocked = int((xk < 0).sum())
    assert 0 < blocked < 16
    assert math.isclose(ao[16, 16, 16], 1.0 - blocked / 16.0, abs_tol=1e-12)


# --- shadow grid: slab on the light's side --------------------------------------------
@pytest.mark.parametrize("rho0", [0.05, 0.5])
def test_shadow_slab_towards_light(rho0):
    """Dense slab 20 <= z < 24, light towards +z, aperture 0 (unit steps
    from the voxel centre land on cell centres, trilinear weight 1). A voxel
    below the slab sees 1 - min(1, rho0 * 4); inside the slab only the slab
    cells above it count; above the slab nothing blocks the light."""
    g = (8, 8, 32)
    lvl0 = np.zeros((32, 8, 8))
    lvl0[20:24] = rho0
    rho = _level0_pyramid(g, lvl0)
    sh = O.shadow_grid(rho, g, (0.0, 0.0, 1.0), aperture=0.0).reshape(32, 8, 8)
    for z in range(32):
        path = max(0, 24 - max(z + 1, 20))        # slab cells strictly above voxel z
        expect = 1.0 - min(1.0, rho0 * path)
        assert np.allclose(sh[z], expect, atol=1e-12), z
    # traced away from the light (towards -z) the slab would shade the voxels above it
    flipped = O.shadow_grid(rho, g, (0.0, 0.0, -1.0), aperture=0.0).reshape(32, 8, 8)
    assert flipped[5, 4, 4] == 1.0 and flipped[28, 4, 4] == pytest.approx(1 - min(1, 4 * rho0))
    assert sh[5, 4, 4] == pytest.approx(1 - min(1, 4 * rho0))


# --- shading 2 closed form --------------------------------------------------------------
def _one_line(grid=16):
    """One straight line along x at y = 8 + 1/64, z = 2 + 33/64 (bin centres
    for N = 32, so the decoded line is exact)."""
    yc = 8 * 256 + 4
    z = 2 * 256 + 128 + 4
    lat = np.array([[256 + 20, yc, z], [256 * (grid - 1) - 20, yc, z]], np.int32)
    return O.voxelize(lat, np.array([0, 2]), None, (grid,) * 3, 32)


def _cam(eye, w=1, h=1):
    return synth.Camera(tuple(map(float, eye)), (0.0, 0.0, -1.0), (0.0, 0.0, 0.0),
                        (0.0, 0.0, 0.0), w, h, True)


@pytest.mark.parametrize("light", [(0.3, 0.4, 0.866), (0.3, 0.4, -0.866), (-0.6, 0.0, 0.8)])
def test_shading2_head_on_closed_form(light):
    """Opaque line, ray straight down through its axis: the entry normal is
    n = +z = v. With AO linear in z and SH constant, the colour is
    base (ka AO(x) + kd SH max(0, n.L)) + ks SH max(0, n.h)^p, h = (L + v)/|L + v|,
    AO taken at the entry point x (z = axis + r)."""
    grid = 16
    csr = _one_line(grid)
    base = np.array([0.5, 0.25, 1.0], np.float32)
    lut = synth.lut_constant(tuple(base), 1.0)
    r = np.float32(0.4)
    yc, zc = 8.0 + 1.0 / 64, 2.0 + 33.0 / 64
    L = np.array(light, np.float32).astype(np.float64)
    L32 = L / np.linalg.norm(L)
    L32 = L32.astype(np.float32)
    Ld = L32.astype(np.float64)
    # AO(z) = 0.2 + 0.1 (z - 0.5) at cell centres, linear in z: trilinear is exact inside
    zz = np.arange(grid)[:, None, None] + 0.5
    ao = np.broadcast_to(0.2 + 0.1 * (zz - 0.5), (grid, grid, grid)).ravel().copy()
    s0 = 0.7
    sh = np.full(grid ** 3, s0)
    ka, kd, ks, p = 0.25, 0.75, 0.2, 16.0
    img, _ = O.render(csr, grid, 32, _cam((6.5, yc, 40.0)), ao=ao, sh=sh, lut=lut,
                      radius=float(r), opaque=True, shading=2, mode=0, ka=ka, kd=kd, ks=ks,
                      shininess=p, light_dir=tuple(float(x) for x in L32))
    x_z = zc + float(r)
    ao_x = 0.2 + 0.1 * (x_z - 0.5)
    v = np.array([0.0, 0.0, 1.0])
    ndl = max(0.0, Ld[2])
    h = (Ld + v) / np.linalg.norm(Ld + v)
    ndh = max(0.0, h[2])
    col = base.astype(np.float64) * (ka * ao_x + kd * s0 * ndl) + ks * s0 * ndh ** p
    assert np.allclose(img[0, 0, :3], col, atol=1e-9), (img[0, 0], col)
    assert img[0, 0, 3] == 1.0
    if light[2] < 0:
        # light from below: the diffuse term vanishes, the ambient term remains
        assert np.allclose(img[0, 0, :3], base * ka * ao_x + ks * s0 * ndh ** p, atol=1e-9)


def test_shading2_transparent_weights():
    """Transparent: the same colour weighted by alpha, premultiplied."""
    grid = 16
    csr = _one_line(grid)
    base = np.array([0.1, 0.9, 0.3], np.float32)
    a = np.float32(0.35)
    lut = synth.lut_constant(tuple(base), float(a))
    ao = np.full(grid ** 3, 0.5)
    sh = np.full(grid ** 3, 0.25)
    L32 = np.array([0.0, 0.6, 0.8], np.float32)
    img, _ = O.render(csr, grid, 32, _cam((6.5, 8.0 + 1.0 / 64, 40.0)), ao=ao, sh=sh, lut=lut,
                      radius=0.4, opaque=False, shading=2, mode=1, alpha_stop=0.95,
                      light_dir=tuple(float(x) for x in L32))
    Ld = L32.astype(np.float64)
    h = (Ld + [0, 0, 1]) / np.linalg.norm(Ld + [0, 0, 1])
    col = base.astype(np.float64) * (0.25 * 0.5 + 0.75 * 0.25 * Ld[2]) + 0.2 * 0.25 * h[2] ** 16
    assert np.allclose(img[0, 0, :3], float(a) * col, atol=1e-9)
    assert math.isclose(img[0, 0, 3], float(a), abs_tol=1e-12)
