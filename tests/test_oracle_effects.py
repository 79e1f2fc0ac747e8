"""Pins for the oracle's optional rendering effects.

Section "Transparency rendering": the opacity of a tube hit can depend on the
distance the ray travels inside the tube. Reading: the transfer function's
opacity is that of a chord of one tube diameter; a chord of length l has
opacity 1 - (1 - alpha)^(l / 2r). Checked with chords the geometry fixes: a
ray through the axis (l = 2r), rays at offset b (l = 2 sqrt(r^2 - b^2)), a
ray along the tube (l = segment length + 2r), and stacks of equal layers.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1801_01155_amd import synth


def _cam(eye, fwd=(0.0, 0.0, -1.0), right=(0.0, 0.0, 0.0), up=(0.0, 0.0, 0.0), w=1, h=1):
    return synth.Camera(tuple(map(float, eye)), tuple(map(float, fwd)), tuple(map(float, right)),
                        tuple(map(float, up)), w, h, True)


def _stack(n, grid=16):
    """n lines along x at y = 8 + 1/64, z = 2.5 + k + 1/64 (bin centres, N = 32)."""
    yc = 8 * 256 + 4
    lat, off = [], [0]
    for k in range(n):
        z = (2 + k) * 256 + 128 + 4
        lat += [[256 + 20, yc, z], [256 * (grid - 1) - 20, yc, z]]
        off.append(len(lat))
    return O.voxelize(np.array(lat, np.int32), np.array(off), None, (grid,) * 3, 32)


YC = 8.0 + 1.0 / 64


@pytest.mark.parametrize("alpha", [0.3, 0.05, 1.0])
def test_chord_through_axis_gives_lut_alpha(alpha):
    csr = _stack(1)
    lut = synth.lut_constant((0.2, 0.4, 0.6), alpha)
    r = 0.4
    for mode in (0, 1):
        img, _ = O.render(csr, 16, 32, _cam((6.5, YC, 40.0)), lut=lut, radius=r, opaque=False,
                          alpha_stop=1.01, shading=0, mode=mode, distance_alpha=True)
        a32 = float(np.float32(alpha))
        assert math.isclose(img[0, 0, 3], a32, abs_tol=1e-12)
        assert np.allclose(img[0, 0, :3], np.array([0.2, 0.4, 0.6], np.float32) * a32, atol=1e-12)


@pytest.mark.parametrize("scale", [1.0, 2.5])
@pytest.mark.parametrize("b", [0.0, 0.1, 0.25, 0.35, 0.399])
def test_chord_at_offset(b, scale):
    csr = _stack(1)
    alpha = 0.4
    lut = synth.lut_constant((1.0, 1.0, 1.0), alpha)
    r = np.float32(0.4)
    y = np.float32(YC + b)
    # the ray direction need not be unit length: the chord is a distance
    img, _ = O.render(csr, 16, 32, _cam((6.5, float(y), 40.0), fwd=(0.0, 0.0, -scale)), lut=lut,
                      radius=float(r), opaque=False, alpha_stop=1.01, shading=0, mode=1,
                      distance_alpha=True)
    bb = float(y) - YC
    chord = 2.0 * math.sqrt(float(r) ** 2 - bb * bb)
    a32 = float(np.float32(alpha))
    expect = 1.0 - (1.0 - a32) ** (chord / (2.0 * float(r)))
    assert math.isclose(img[0, 0, 3], expect, rel_tol=1e-9, abs_tol=1e-12)
    # constant opacity ignores the chord
    img, _ = O.render(csr, 16, 32, _cam((6.5, float(y), 40.0)), lut=lut, radius=float(r),
                      opaque=False, alpha_stop=1.01, shading=0, mode=1, distance_alpha=False)
    assert math.isclose(img[0, 0, 3], a32, abs_tol=1e-12)


def test_chord_along_the_tube():
    """A ray along a single straight segment inside one voxel travels its
    length plus one radius into each end sphere."""
    grid = 8
    # one line along x inside voxel (3, 4, 4): from the -x face to the +x face
    lat = np.array([[2 * 256 + 128, 4 * 256 + 132, 4 * 256 + 132],
                    [5 * 256 + 128, 4 * 256 + 132, 4 * 256 + 132]], np.int32)
    csr = O.voxelize(lat, np.array([0, 2]), None, (grid,) * 3, 32)
    assert len(csr.records) == 2                        # voxels 3 and 4
    alpha = 0.2
    lut = synth.lut_constant((1.0, 1.0, 1.0), alpha)
    r = float(np.float32(0.3))
    yz = 4.0 + 16.5 / 32                                 # bin 16 centre
    cam = _cam((-5.0, yz, yz), fwd=(1.0, 0.0, 0.0))
    img, _ = O.render(csr, grid, 32, cam, lut=lut, radius=r, opaque=False, alpha_stop=1.01,
                      shading=0, mode=1, merge_curves=True, distance_alpha=True)
    # the first capsule (voxel 3, x in [3, 4]) is composited with its own chord
    # 1 + 2r; the second overlaps it at the joint and merges
    a32 = float(np.float32(alpha))
    expect = 1.0 - (1.0 - a32) ** ((1.0 + 2.0 * r) / (2.0 * r))
    assert math.isclose(img[0, 0, 3], expect, rel_tol=1e-9)


@pytest.mark.parametrize("n,alpha", [(3, 0.3), (7, 0.1)])
def test_distance_alpha_stack_head_on(n, alpha):
    csr = _stack(n, grid=16)
    lut = synth.lut_constant((0.5, 0.5, 0.5), alpha)
    img, _ = O.render(csr, 16, 32, _cam((6.5, YC, 40.0)), lut=lut, radius=0.4, opaque=False,
                      alpha_stop=1.01, shading=0, mode=1, distance_alpha=True)
    a32 = float(np.float32(alpha))
    assert math.isclose(img[0, 0, 3], 1 - (1 - a32) ** n, abs_tol=1e-12)


def test_distance_alpha_opaque_unchanged():
    csr = _stack(1)
    lut = synth.lut_constant((0.5, 0.25, 1.0), 1.0)
    for y in (YC, YC + 0.39):
        a, _ = O.render(csr, 16, 32, _cam((6.5, y, 40.0)), lut=lut, radius=0.4, opaque=True,
                        shading=1, distance_alpha=True)
        b, _ = O.render(csr, 16, 32, _cam((6.5, y, 40.0)), lut=lut, radius=0.4, opaque=True,
                        shading=1, distance_alpha=False)
        assert np.array_equal(a, b) and a[0, 0, 3] == 1.0
