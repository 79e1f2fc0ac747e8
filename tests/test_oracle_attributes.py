"""Pins for per-vertex attributes (section "Curve voxelization": line
attributes interpolated to the line-face intersection points; section
"Illumination effects": without interpolation the colours show steps at the
voxel boundaries).

Each event on segment v_i -> v_{i+1} gets a_i + (a_{i+1} - a_i) t rounded
half up (t the exact parameter of the face crossing); each line keeps its two
endpoint attributes, its record's attribute byte is their mean rounded down;
a fragment's colour and opacity come from the transfer function read
linearly at the attribute interpolated along the line at the segment point
closest to the entry point. Checked against closed forms and an
exact-rational brute force; each pin fails under a plausible slip (rounding
down instead of half up, the parameter taken from the other end, the
record's mean attribute or the nearest transfer-function entry used for the
fragment)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1801_01155_amd import synth
from tests.brute import vox_fraction as BF


def _x_line(attrs=(0, 255), y=2 * 256 + 132, z=2 * 256 + 132):
    """One segment along x from x = 0.5 to x = 3.5 voxels in a 5^3 grid."""
    lat = np.array([[128, y, z], [3 * 256 + 128, y, z]], np.int32)
    return O.voxelize(lat, np.array([0, 2]), None, (5, 5, 5), 32, vattr=np.array(attrs, np.uint8))


def test_event_attributes_closed_form():
    # crossings of x = 1, 2, 3 at t = 1/6, 1/2, 5/6: 42.5, 127.5, 212.5 -> 43, 128, 213
    csr = _x_line()
    assert len(csr.records) == 2
    assert csr.ends.tolist() == [43 | (128 << 8), 128 | (213 << 8)]
    # record attribute bytes: the mean rounded down, (43 + 128) // 2, (128 + 213) // 2
    assert [(int(r) >> 32) & 0xFF for r in csr.records] == [85, 170]
    # a decreasing ramp: 255 - 42.5 = 212.5 -> 213, 127.5 -> 128, 42.5 -> 43
    down = _x_line((255, 0))
    assert down.ends.tolist() == [213 | (128 << 8), 128 | (43 << 8)]


def test_attributes_inside_one_voxel_do_not_leak():
    # the attribute changes over a segment that stays inside voxel 1; the
    # crossing of x = 2 happens on the next segment, from its own endpoints
    y = z = 2 * 256 + 132
    lat = np.array([[128, y, z], [300, y, z], [400, y, z], [3 * 256 + 128, y, z]], np.int32)
    csr = O.voxelize(lat, np.array([0, 4]), None, (5, 5, 5), 32,
                     vattr=np.array([10, 20, 200, 100], np.uint8))
    # x = 256 on segment 0 at t = 128/172: 10 + 10 * 128/172 = 17.44 -> 17;
    # x = 512 on segment 2 at t = 112/496: 200 - 100 * 112/496 = 177.42 -> 177;
    # x = 768 at t = 368/496: 200 - 100 * 368/496 = 125.8 -> 126
    assert csr.ends.tolist() == [17 | (177 << 8), 177 | (126 << 8)]


@pytest.mark.parametrize("seed,step,bins", [(1, 64, 4), (2, 7, 32), (3, 1, 8)])
def test_attributes_match_fraction_bruteforce(seed, step, bins):
    rng = np.random.default_rng(seed)
    grid = (5, 4, 6)
    verts, off = [], [0]
    for _ in range(50):
        n = int(rng.integers(2, 10))
        p = rng.integers(1, np.array(grid) - 1) * 256 + rng.integers(0, 256 // step, 3) * step
        pts = [p]
        for _ in range(n - 1):
            pts.append(np.clip(pts[-1] + rng.integers(-2 * 256 // step, 2 * 256 // step + 1, 3) * step,
                               0, np.array(grid) * 256 - 1))
        verts += pts
        off.append(len(verts))
    lat = np.array(verts, np.int32)
    off = np.array(off, np.int64)
    va = rng.integers(0, 256, len(lat)).astype(np.uint8)
    got = O.voxelize(lat, off, None, grid, bins, vattr=va)
    offs, recs, ends = BF.voxelize(lat, off, None, grid, bins, vattr=va)
    assert got.offsets.tolist() == offs
    assert got.records.tolist() == recs
    assert got.ends.tolist() == ends
    # without vertex attributes the geometry is the same
    plain = O.voxelize(lat, off, None, grid, bins)
    assert np.array_equal(plain.records & np.uint64(0x3FFFFFFF), got.records & np.uint64(0x3FFFFFFF))


def _lut_linear():
    x = np.arange(256, dtype=np.float64)
    lut = np.zeros((256, 4), np.float32)
    lut[:, 0] = x / 255.0
    lut[:, 1] = 1.0 - x / 255.0
    lut[:, 2] = 0.5
    lut[:, 3] = 0.1 + 0.8 * x / 255.0
    return lut


@pytest.mark.parametrize("xh,opaque", [(1.25, True), (1.625, False), (2.5, True)])
def test_fragment_colour_interpolated_along_the_line(xh, opaque):
    """A ray straight down onto the line at x = xh: the entry point's closest
    segment point lies at x = xh, so u = frac(xh) of the voxel's line from
    x = floor(xh) to floor(xh) + 1; the attribute is e + u (x - e) and the
    colour the transfer function read linearly there."""
    csr = _x_line()
    lut = _lut_linear()
    yc = 2 + (16 + 0.5) / 32   # y bin 16 of 32 (lattice 132/256 -> bin 16)
    cam = synth.Camera((xh, yc, 10.0), (0.0, 0.0, -1.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0),
                       1, 1, True)
    img, _ = O.render(csr, (5, 5, 5), 32, cam, lut=lut, radius=0.3, opaque=opaque, shading=0,
                      mode=0, alpha_stop=0.95)
    if xh < 2:
        e, x, u = 43.0, 128.0, xh - 1.0
    else:
        e, x, u = 128.0, 213.0, xh - 2.0
    af = e + u * (x - e)
    i0 = int(math.floor(af))
    f = af - i0
    col = (1 - f) * lut[i0].astype(np.float64) + f * lut[i0 + 1].astype(np.float64)
    a = 1.0 if opaque else col[3]
    assert np.allclose(img[0, 0, :3], a * col[:3], atol=1e-9), (img[0, 0], col, a)
    assert math.isclose(img[0, 0, 3], a, abs_tol=1e-9)
    # not the record's mean attribute, nor the nearest entry
    mean = int(csr.records[0 if xh < 2 else 1] >> np.uint64(32)) & 0xFF
    assert abs(img[0, 0, 0] - a * lut[mean, 0]) > 1e-4


def test_density_uses_the_mean_attribute():
    csr = _x_line()
    lut = _lut_linear()
    _, _, rho, _, _ = O.lod(csr, (5, 5, 5), 32, lut, opaque=False)
    # voxel (1, 2, 2): one line of length 1 with attribute byte 85
    v = 1 + 5 * (2 + 5 * 2)
    assert rho[v] == pytest.approx(float(lut[85, 3]), abs=1e-12)
