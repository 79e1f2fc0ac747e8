"""Pins for the oracle's ray set-up, grid walk, ray-tube test and compositing.

Sections "Line Raycasting", "Ray-tube intersections", "Rendering effects" and
"Transparency rendering". Checked against brute force over all capsules,
textbook special cases and closed forms for uniform-opacity stacks.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests.brute import render_brute as RB
from paper_1801_01155_amd import synth


def _cam(eye, fwd, right, up, w, h, ortho):
    return synth.Camera(tuple(map(float, eye)), tuple(map(float, fwd)), tuple(map(float, right)),
                        tuple(map(float, up)), w, h, ortho)


# --- ray per pixel -----------------------------------------------------------------
@pytest.mark.parametrize("ortho", [False, True])
def test_ray_contract(ortho):
    cam = synth.default_camera((64, 64, 64), 37, 23, orthographic=ortho)
    for (i, j) in [(0, 0), (36, 22), (5, 17), (18, 11)]:
        o, d = O.ray(cam, i, j)
        ro, rd = RB.ray_for_pixel(cam, i, j)
        assert np.array_equal(o.astype(np.float64), ro) and np.array_equal(d.astype(np.float64), rd)
    # the centre pixel of an odd image looks along forward
    cam = synth.default_camera((64, 64, 64), 5, 5, orthographic=ortho)
    o, d = O.ray(cam, 2, 2)
    assert np.allclose(d, cam.forward, atol=1e-7)


# --- grid walk -----------------------------------------------------------------------
def _brute_voxels(grid, o, d):
    o = o.astype(np.float64)
    d = d.astype(np.float64)
    out = []
    for z in range(grid[2]):
        for y in range(grid[1]):
            for x in range(grid[0]):
                lo, hi = 0.0, np.inf
                ok = True
                for a, c in enumerate((x, y, z)):
                    if d[a] != 0:
                        ta, tb = (c - o[a]) / d[a], (c + 1 - o[a]) / d[a]
                        lo, hi = max(lo, min(ta, tb)), min(hi, max(ta, tb))
                    elif not (c <= o[a] < c + 1):
                        ok = False
                if ok and lo < hi:
                    out.append((lo, hi, (x, y, z)))
    out.sort()
    return out


@pytest.mark.parametrize("seed", range(6))
def test_dda_matches_bruteforce(seed):
    rng = np.random.default_rng(seed)
    grid = (7, 5, 6)
    for _ in range(40):
        o = (rng.uniform(-6, 12, 3)).astype(np.float32)
        d = rng.normal(size=3).astype(np.float32)
        if seed % 3 == 0:
            d[rng.integers(0, 3)] = 0.0          # axis-parallel component
        cells, t0, t1 = O.dda(grid, o, d)
        ref = _brute_voxels(grid, o, d)
        assert [tuple(c) for c in cells] == [r[2] for r in ref]
        if len(ref):
            assert np.allclose(t0, [r[0] for r in ref], rtol=0, atol=1e-9)
            assert np.allclose(t1, [r[1] for r in ref], rtol=0, atol=1e-9)
            assert (np.diff(t0) > 0).all()
            assert np.array_equal(t0[1:], t1[:-1])                # contiguous
            assert (np.abs(np.diff(cells, axis=0)).sum(1) == 1).all()  # 6-connected


def test_dda_tie_goes_to_lowest_axis():
    # a ray exactly through the x/y edges: steps x first, visiting an empty interval
    cells, t0, t1 = O.dda((4, 4, 1), np.array([0.5, 0.5, 0.5], np.float32),
                          np.array([1, 1, 0], np.float32))
    assert [tuple(c) for c in cells[:3]] == [(0, 0, 0), (1, 0, 0), (1, 1, 0)]
    assert t0[1] == t1[1]


# --- ray vs capsule ------------------------------------------------------------------
def test_capsule_perpendicular_chord():
    r = 0.4
    hit = O.capsule([0.5, -5, 0.3], [0, 2, 0], [0, 0, 0.3], [1, 0, 0.3], r)
    assert hit is not None
    ti, to, n = hit
    assert math.isclose((to - ti) * 2.0, 2 * r, abs_tol=1e-12)
    assert math.isclose(ti, (5 - r) / 2, abs_tol=1e-12)
    assert np.allclose(n, [0, -1, 0])


def test_capsule_offset_chord_and_depth():
    r, b = 0.4, 0.25
    ti, to, _ = O.capsule([0.5, -3, b], [0, 1, 0], [0, 0, 0], [1, 0, 0], r)
    assert math.isclose(ti, 3 - math.sqrt(r * r - b * b), abs_tol=1e-12)
    assert math.isclose(to - ti, 2 * math.sqrt(r * r - b * b), abs_tol=1e-12)
    assert O.capsule([0.5, -3, r + 1e-6], [0, 1, 0], [0, 0, 0], [1, 0, 0], r) is None


def test_capsule_along_axis_hits_spheres():
    r = 0.3
    ti, to, n = O.capsule([-2, 0, 0], [1, 0, 0], [0, 0, 0], [1, 0, 0], r)
    assert math.isclose(ti, 2 - r, abs_tol=1e-12) and math.isclose(to, 3 + r, abs_tol=1e-12)
    assert np.allclose(n, [-1, 0, 0])
    # parallel but off-axis by b < r: enters sphere A off its pole
    b = 0.2
    ti, _, _ = O.capsule([-2, b, 0], [1, 0, 0], [0, 0, 0], [1, 0, 0], r)
    assert math.isclose(ti, 2 - math.sqrt(r * r - b * b), abs_tol=1e-12)


def test_capsule_matches_numeric_root_finding():
    rng = np.random.default_rng(7)
    n_hit = 0
    for _ in range(300):
        a, b = rng.uniform(0, 1, 3), rng.uniform(0, 1, 3)
        o = rng.uniform(-3, 4, 3)
        tgt = rng.uniform(-0.2, 1.2, 3)
        d = tgt - o
        r = rng.uniform(0.05, 0.5)
        h = O.capsule(o, d, a, b, r)
        hit, ti, to = RB.capsule_intervals(o, d, a[None], b[None], r, -10.0, 10.0)
        assert (h is not None) == bool(hit[0])
        if h is not None:
            n_hit += 1
            assert abs(h[0] - ti[0]) < 1e-9 and abs(h[1] - to[0]) < 1e-9
            P = o + h[0] * d
            ba = b - a
            u = np.clip((P - a) @ ba / (ba @ ba), 0, 1)
            assert math.isclose(np.linalg.norm(P - (a + u * ba)), r, rel_tol=1e-9)
    assert n_hit > 50


# --- exact mode == brute force over all capsules -------------------------------------
def _tiny_set(seed, grid, n_curves, n_vert):
    rng = np.random.default_rng(seed)
    verts, off = [], [0]
    for _ in range(n_curves):
        p = rng.uniform(256 * 1.2, 256 * (np.array(grid) - 1.2))
        pts = [p]
        for _ in range(n_vert - 1):
            p = np.clip(p + rng.normal(size=3) * 160, 256 * 1.05, 256 * (np.array(grid) - 1.05))
            pts.append(p)
        verts += [np.floor(q).astype(np.int32) for q in pts]
        off.append(len(verts))
    attr = rng.integers(0, 256, n_curves).astype(np.uint8)
    return np.array(verts, dtype=np.int32), np.array(off, dtype=np.int64), attr


@pytest.mark.parametrize("seed,opaque,shading", [(1, False, 1), (2, True, 1), (3, False, 0),
                                                 (4, False, 1)])
def test_exact_mode_equals_bruteforce(seed, opaque, shading):
    grid = (6, 5, 7)
    lat, off, attr = _tiny_set(seed, grid, 6, 10)
    csr = O.voxelize(lat, off, attr, grid, 16)
    assert len(csr.records) > 10
    lut = synth.lut_importance_alpha(0.15, 0.6)
    cam = synth.orbit_cameras(grid, 1, seed, 24, 20, orthographic=bool(seed % 2))[0]
    kw = dict(radius=0.35, opaque=opaque, alpha_stop=0.95, merge_curves=True, shading=shading)
    img, cnt = O.render(csr, grid, 16, cam, mode=1, lut=lut, **kw)
    ref = RB.render(csr.offsets, csr.records, grid, 16, cam, lut, **kw)
    assert cnt["fragments"] > 10
    err = np.abs(img.reshape(-1, 4) - ref).max(1)
    # numeric roots lose precision only at grazing hits (f ~ (t - t*)^2)
    assert err.max() < 1e-5 and (err > 1e-7).mean() < 0.01


@pytest.mark.parametrize("seed,opaque,shading", [(1, False, 1), (2, True, 1), (5, False, 0),
                                                 (6, False, 1)])
def test_own_voxel_mode_equals_bruteforce(seed, opaque, shading):
    # the own-voxel (fast) mode against its definition written without a grid
    # walk: voxels by brute-force box tests, their own lines' hits (t_in >= 0)
    # composited voxel by voxel; tubes wide enough to leave their voxels
    grid = (6, 5, 7)
    lat, off, attr = _tiny_set(seed, grid, 6, 10)
    csr = O.voxelize(lat, off, attr, grid, 16)
    lut = synth.lut_importance_alpha(0.15, 0.6)
    cam = synth.orbit_cameras(grid, 1, seed, 24, 20, orthographic=bool(seed % 2))[0]
    kw = dict(radius=0.35, opaque=opaque, alpha_stop=0.95, merge_curves=True, shading=shading)
    img, cnt = O.render(csr, grid, 16, cam, mode=0, lut=lut, **kw)
    ref = RB.render_own_voxel(csr.offsets, csr.records, grid, 16, cam, lut, **kw)
    assert cnt["fragments"] > 10
    err = np.abs(img.reshape(-1, 4) - ref).max(1)
    assert err.max() < 1e-5 and (err > 1e-7).mean() < 0.01
    # here the own-voxel order is not the exact one, so the pin tells them apart
    exact, _ = O.render(csr, grid, 16, cam, mode=1, lut=lut, **kw)
    assert np.abs(img - exact).max() > 1e-3


def test_fast_equals_exact_for_thin_separated_tubes():
    # thin tubes never leave their own voxel, so own-voxel lists are complete
    grid = (6, 6, 6)
    lat, off, attr = _tiny_set(11, grid, 5, 12)
    csr = O.voxelize(lat, off, attr, grid, 32)
    lut = synth.lut_importance_alpha(0.2, 0.6)
    cam = synth.orbit_cameras(grid, 1, 3, 32, 32)[0]
    kw = dict(radius=0.01, opaque=False, alpha_stop=0.99, merge_curves=True, shading=1, lut=lut)
    a, _ = O.render(csr, grid, 32, cam, mode=0, **kw)
    b, _ = O.render(csr, grid, 32, cam, mode=1, **kw)
    assert np.abs(a - b).max() < 1e-12


# --- compositing closed forms ----------------------------------------------------------
def _stack(n, alpha, grid=16, bins=32):
    """n straight lines along x at y = 8 + 0.5/N, z = 2, 3, ..., stacked in z."""
    lat, off = [], [0]
    yc = 8 * 256 + 4                          # centre of bin 0 for N = 32
    for k in range(n):
        z = (2 + k) * 256 + 128 + 4           # centre of bin 16
        lat += [[256 + 20, yc, z], [256 * (grid - 1) - 20, yc, z]]
        off.append(len(lat))
    lut = synth.lut_constant((0.2, 0.6, 0.9), alpha)
    csr = O.voxelize(np.array(lat, np.int32), np.array(off), None, (grid,) * 3, bins)
    return csr, lut


@pytest.mark.parametrize("n,alpha,tau", [(5, 0.3, 1.01), (9, 0.2, 0.95), (12, 0.5, 0.95),
                                         (6, 0.1, 1.01)])
def test_uniform_alpha_stack_closed_form(n, alpha, tau):
    grid = 16
    csr, lut = _stack(n, alpha, grid)
    # orthographic, looking down -z through the stack
    cam = _cam((5.3, 8.0 + 0.5 / 32, 40.0), (0, 0, -1), (0.5, 0, 0), (0, 0.5, 0), 9, 9, True)
    for mode in (0, 1):
        img, _ = O.render(csr, grid, 32, cam, mode=mode, lut=lut, radius=0.4, opaque=False,
                          alpha_stop=tau, merge_curves=True, shading=0)
        centre = img[4, 4]
        alpha = float(np.float32(alpha))       # the transfer function holds fp32
        k = n if tau > 1 else min(n, math.ceil(math.log(1 - tau) / math.log(1 - alpha)))
        A = 1 - (1 - alpha) ** k
        assert math.isclose(centre[3], A, abs_tol=1e-12)
        assert np.allclose(centre[:3], np.array([0.2, 0.6, 0.9], np.float32) * A, atol=1e-7)


def test_merge_blends_each_curve_once():
    # the ray crosses one voxel boundary of each line, where two capsules of the
    # same curve overlap; with merging it is blended once, without it twice
    grid = 16
    csr, lut = _stack(3, 0.3, grid)
    cam = _cam((4.0, 8.0 + 0.5 / 32, 40.0), (0, 0, -1), (0.01, 0, 0), (0, 0.01, 0), 1, 1, True)
    kw = dict(lut=lut, radius=0.4, opaque=False, alpha_stop=1.01, shading=0, mode=1)
    m, _ = O.render(csr, grid, 32, cam, merge_curves=True, **kw)
    u, _ = O.render(csr, grid, 32, cam, merge_curves=False, **kw)
    a = float(np.float32(0.3))
    assert math.isclose(m[0, 0, 3], 1 - (1 - a) ** 3, abs_tol=1e-12)
    assert math.isclose(u[0, 0, 3], 1 - (1 - a) ** 6, abs_tol=1e-12)


def test_opaque_first_hit_shading_and_coverage():
    grid = 16
    csr, _ = _stack(1, 1.0, grid)
    lut = synth.lut_constant((0.5, 0.25, 1.0), 1.0)
    r = 0.4
    yc = 8.0 + 0.5 / 32
    # perpendicular ray through the axis: n . v = 1 -> base * (ka + kd) + ks
    cam = _cam((6.5, yc, 40.0), (0, 0, -1), (0.0, 0, 0), (0, 0.0, 0), 1, 1, True)
    img, _ = O.render(csr, grid, 32, cam, lut=lut, radius=r, opaque=True, shading=1, mode=0)
    assert np.allclose(img[0, 0], [0.5 * 1.0 + 0.2, 0.25 + 0.2, 1.0 + 0.2, 1.0], atol=1e-7)
    # coverage: a pixel is covered iff its ray passes within r of the axis
    W = 41
    cam = _cam((6.5, yc, 40.0), (0, 0, -1), (0.0, 0, 0), (0, 1.0, 0), 1, W, True)
    # (neighbour-voxel mode: below y = 8 the tube lies in voxels that do not own it)
    img, _ = O.render(csr, grid, 32, cam, lut=lut, radius=r, opaque=True, shading=0, mode=1)
    for j in range(W):
        v = 1.0 - 2.0 * (j + 0.5) / W
        y = np.float32(np.float32(yc) + v * 1.0)
        inside = abs(float(y) - yc) < r - 1e-9
        outside = abs(float(y) - yc) > r + 1e-9
        if inside:
            assert img[j, 0, 3] == 1.0
        if outside:
            assert img[j, 0, 3] == 0.0


def test_counters_consistent():
    grid = (6, 5, 7)
    lat, off, attr = _tiny_set(5, grid, 6, 10)
    csr = O.voxelize(lat, off, attr, grid, 16)
    cam = synth.orbit_cameras(grid, 1, 9, 16, 16)[0]
    lut = synth.lut_importance_alpha()
    _, k = O.render(csr, grid, 16, cam, mode=0, lut=lut, opaque=False, merge_curves=True)
    assert k["visited"] >= k["nonempty"] and k["tested"] >= k["hits"] >= k["fragments"] > 0


def _golden_rows(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = []
    for line in open(path):
        line = line.split("#", 1)[0].split()
        if line:
            rows.append(line)
    return rows


@pytest.mark.parametrize("row", _golden_rows("uniform_slab.txt"), ids=lambda r: "_".join(r[:2]))
def test_uniform_slab_golden(row):
    """Uniform-opacity layers against the closed-form values stored in
    tests/golden/uniform_slab.txt, without and with alpha-termination."""
    a, n, A_n, n_star = float(row[0]), int(row[1]), float(row[2]), int(row[3])
    a32 = float(np.float32(a))
    for layers, tau, expect_k in ((n, 1.01, n), (n_star + 3, 0.95, n_star)):
        grid = max(16, layers + 4)
        csr, lut = _stack(layers, a, grid)
        cam = _cam((5.3, 8.0 + 0.5 / 32, grid + 10.0), (0, 0, -1), (0.5, 0, 0), (0, 0.5, 0),
                   9, 9, True)
        img, _ = O.render(csr, grid, 32, cam, mode=1, lut=lut, radius=0.4, opaque=False,
                          alpha_stop=tau, merge_curves=True, shading=0)
        A = img[4, 4, 3]
        if layers == n:
            # the table's decimal value; the LUT holds alpha rounded to fp32
            assert abs(A - A_n) < 2e-7 * n
        assert math.isclose(A, 1 - (1 - a32) ** expect_k, abs_tol=1e-12)
