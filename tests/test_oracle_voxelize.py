"""Pins for the oracle's grid set-up and voxelizer (CPU only).

Sections "Curve voxelization", "Line quantization", "GPU implementation" and
"Memory statistics". The oracle is checked against an exact-rational
brute force, hand-derived closed forms and invariants the paper states.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests.brute import vox_fraction as BF
from paper_1801_01155_amd import synth


def _code(face, bu, bw):
    return face | (bu << 3) | (bw << 9)


def _rec(entry, exit_, attr=255, curve=0):
    return entry | (exit_ << 15) | (attr << 32) | (curve << 40)


# --- Memory statistics: bytes per line as printed (tests/golden/record_bytes.txt)
def test_paper_record_bytes():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "record_bytes.txt")
    rows = [l.split("#", 1)[0].split() for l in open(path)]
    rows = [r for r in rows if r and r[0] != "header_bytes"]
    assert len(rows) == 6
    for n, nbytes, bin_bits in rows:
        n = int(n)
        assert O.paper_record_bytes(n) == int(nbytes)
        assert 2 * int(math.log2(n)) == int(bin_bits)


# --- Curve voxelization, grid set-up ------------------------------------------------
def test_grid_setup_bbox_and_aspect():
    rng = np.random.default_rng(0)
    xyz = (rng.normal(size=(500, 3)) * [3.0, 1.0, 0.5] + [10, -4, 2]).astype(np.float32)
    R = 64
    lat, lo, s = O.grid_setup(xyz, R)
    ext = xyz.astype(np.float64).max(0) - xyz.astype(np.float64).min(0)
    assert np.allclose(lo, xyz.min(0))
    # the longest extent spans exactly R - 2 voxels, starting one voxel in
    assert lat.min(0).tolist() == [256, 256, 256]
    assert lat[:, 0].max() == 256 * (R - 1)
    # aspect ratio kept to lattice rounding
    span = lat.max(0) - lat.min(0)
    assert np.allclose(span / span[0], ext / ext[0], atol=2.0 / span[0])
    assert (lat < 256 * R).all() and (lat >= 0).all()
    # rounding to nearest lattice point
    ref = np.floor((xyz.astype(np.float64) - lo) * s + 0.5) + 256
    assert (ref == lat).all()


def test_grid_setup_degenerate():
    lat, lo, s = O.grid_setup(np.ones((4, 3), dtype=np.float32), 8)
    assert s == 0.0 and (lat == 256).all()


# --- Voxelizer vs exact-rational brute force ---------------------------------------
def _random_curves(rng, n_curves, grid, step):
    verts, off = [], [0]
    for _ in range(n_curves):
        n = int(rng.integers(1, 12))
        p = rng.integers(1, np.array(grid) - 1) * 256 + rng.integers(0, 256 // step, 3) * step
        pts = [p.copy()]
        for _ in range(n - 1):
            kind = rng.integers(0, 6)
            if kind == 0 and len(pts) >= 2:
                q = pts[-2].copy()                     # backtrack onto the previous vertex
            elif kind == 1:
                q = pts[-1].copy()                     # zero-length segment
            else:
                q = pts[-1] + rng.integers(-2 * 256 // step, 2 * 256 // step + 1, 3) * step
            q = np.clip(q, 0, np.array(grid) * 256 - 1)
            pts.append(q)
        verts += pts
        off.append(len(verts))
    return np.array(verts, dtype=np.int32), np.array(off, dtype=np.int64)


@pytest.mark.parametrize("seed,step,bins", [(1, 64, 4), (2, 32, 32), (3, 1, 8), (4, 128, 64),
                                            (5, 16, 1), (6, 7, 16)])
def test_voxelize_matches_fraction_bruteforce(seed, step, bins):
    rng = np.random.default_rng(seed)
    grid = (5, 4, 6)
    lat, off = _random_curves(rng, 60, grid, step)
    attr = rng.integers(0, 256, len(off) - 1).astype(np.uint8)
    got = O.voxelize(lat, off, attr, grid, bins)
    offs, recs = BF.voxelize(lat, off, attr, grid, bins)
    assert got.offsets.tolist() == offs
    assert got.records.tolist() == recs


def test_axis_parallel_line_closed_form():
    # y_local = 100/256 -> bin floor(100 * 32 / 256) = 12; z_local = 128/256 -> 16
    lat = np.array([[128, 356, 128], [128 + 3 * 256, 356, 128]], dtype=np.int32)
    csr = O.voxelize(lat, np.array([0, 2]), None, (4, 2, 1), 32)
    # events at x = 256, 512, 768 -> lines in voxels (1,1,0) and (2,1,0)
    rec = _rec(_code(0, 12, 16), _code(1, 12, 16))
    assert csr.records.tolist() == [rec, rec]
    assert np.diff(csr.offsets.astype(int)).nonzero()[0].tolist() == [1 + 4 * 1, 2 + 4 * 1]


def test_edge_event_single_face_lowest_axis():
    # through the x/y edge at (256, 256): one event, face from axis x
    lat = np.array([[128, 128, 128], [384, 384, 128], [640, 384, 128]], dtype=np.int32)
    csr = O.voxelize(lat, np.array([0, 3]), None, (3, 2, 1), 32)
    # events: (256,256) edge: exit (0,0,0) +x, enter (1,1,0) -x with y bin 0;
    #         (512, 384) face: exit (1,1,0) +x with y local 128 -> 16
    assert csr.n_events == 2
    assert csr.records.tolist() == [_rec(_code(0, 0, 16), _code(1, 16, 16))]
    assert csr.offsets[1 + 3 * 1 + 1] - csr.offsets[1 + 3 * 1] == 1


def test_corner_event():
    lat = np.array([[128, 128, 128], [384, 384, 384], [384, 384, 700]], dtype=np.int32)
    csr = O.voxelize(lat, np.array([0, 3]), None, (2, 2, 3), 8)
    # corner (256,256,256): exit (0,0,0) via +x, enter (1,1,1) via -x at (y,z) local (0,0)
    # then z = 512 crossing: exit (1,1,1) via +z at (x,y) local (128,128) -> bins (4,4)
    assert csr.n_events == 2
    assert csr.records.tolist() == [_rec(_code(0, 0, 0), _code(5, 4, 4))]


def test_in_face_segment():
    # a segment lying in the plane x = 256 belongs to voxel x = 1 (half-open)
    lat = np.array([[256, 128, 128], [256, 700, 128]], dtype=np.int32)
    csr = O.voxelize(lat, np.array([0, 2]), None, (3, 3, 1), 32)
    # events at y = 256 and 512; the line in voxel (1,1,0) has x local 0 -> bin 0
    assert csr.records.tolist() == [_rec(_code(2, 0, 16), _code(3, 0, 16))]


def test_touch_and_return_dropped():
    lat = np.array([[128, 128, 128], [256, 128, 128], [128, 128, 128]], dtype=np.int32)
    csr = O.voxelize(lat, np.array([0, 3]), None, (2, 1, 1), 32)
    assert csr.n_events == 2 and csr.n_dropped == 1 and len(csr.records) == 0


def test_short_curves_contribute_nothing():
    lat = np.array([[300, 300, 300], [300, 300, 300], [310, 320, 330]], dtype=np.int32)
    csr = O.voxelize(lat, np.array([0, 1, 1, 3]), None, (4, 4, 4), 32)
    assert len(csr.records) == 0 and csr.offsets[-1] == 0


def test_out_of_range_rejected():
    lat = np.array([[0, 0, 0], [256 * 4, 0, 0]], dtype=np.int32)
    with pytest.raises(ValueError):
        O.voxelize(lat, np.array([0, 2]), None, (4, 4, 4), 32)
    with pytest.raises(ValueError):
        O.voxelize(lat[:1], np.array([0, 1]), None, (4, 4, 4), 24)


# --- Invariants on the small streamline workload ------------------------------------
@pytest.fixture(scope="module")
def small():
    w = synth.WORKLOADS["small"]
    ls = synth.abc_lineset(w["n_curves"], w["n_vertices"], w["seed"])
    lat, _, _ = O.grid_setup(ls.xyz, w["grid"])
    csr = O.voxelize(lat, ls.curve_off, ls.attr, w["grid"], w["bins"])
    return w, ls, lat, csr


def test_small_matches_bruteforce_subset(small):
    w, ls, lat, csr = small
    sub = 40
    off = ls.curve_off[:sub + 1]
    a = O.voxelize(lat[:off[-1]], off, ls.attr[:sub], w["grid"], w["bins"])
    offs, recs = BF.voxelize(lat[:off[-1]], off, ls.attr[:sub], (w["grid"],) * 3, w["bins"])
    assert a.offsets.tolist() == offs and a.records.tolist() == recs


def test_small_csr_invariants(small):
    w, ls, lat, csr = small
    R, N = w["grid"], w["bins"]
    offs = csr.offsets.astype(np.int64)
    assert (np.diff(offs) >= 0).all() and offs[0] == 0 and offs[-1] == len(csr.records)
    # within a voxel: ordered by curve id
    tags = (csr.records >> np.uint64(40)).astype(np.int64)
    owner = np.repeat(np.arange(R ** 3), np.diff(offs))
    key = owner * (1 << 24) + tags
    assert (np.diff(key) >= 0).all()
    # quantized endpoints are bin centres on faces of their own voxel and differ
    for rec in csr.records[:2000]:
        a, b = O.decode(int(rec), N)
        for p in (a, b):
            on_face = [(x == 0.0 or x == 1.0) for x in p]
            assert sum(on_face) == 1
        assert not np.array_equal(a, b)
    # attribute byte and curve tag carried through
    assert set(((csr.records >> np.uint64(32)) & np.uint64(0xFF)).tolist()) <= set(ls.attr.tolist())


def test_small_deviation_and_continuity(small):
    """Deviation bound (section "Curve voxelization": at most a voxel diagonal)
    and joint continuity of consecutive lines of a curve across face events."""
    w, ls, lat, csr = small
    R, N = w["grid"], w["bins"]
    offs = csr.offsets.astype(np.int64)
    owner = np.repeat(np.arange(R ** 3), np.diff(offs))
    tags = (csr.records >> np.uint64(40)).astype(np.int64)
    for c in range(0, 30):
        ks = np.nonzero(tags == c)[0]
        # per-voxel order was (curve, ordinal) -> recover the curve order by walking
        segs = []
        for k in ks:
            v = owner[k]
            cell = np.array([v % R, (v // R) % R, v // (R * R)], dtype=float)
            a, b = O.decode(int(csr.records[k]), N)
            segs.append((cell + a, cell + b, cell))
        verts = lat[ls.curve_off[c]:ls.curve_off[c + 1]] / 256.0
        for a, b, cell in segs:
            inside = np.all((verts >= cell) & (verts <= cell + 1), axis=1)
            for p in verts[inside]:
                ba = b - a
                u = np.clip((p - a) @ ba / (ba @ ba), 0, 1)
                assert np.linalg.norm(p - (a + u * ba)) <= math.sqrt(3) + 1e-9
        # continuity: every exit point that is not on an edge is some line's entry
        entries = {tuple(np.round(a, 9)) for a, _, _ in segs}
        starts = 0
        for a, b, cell in segs:
            if tuple(np.round(b, 9)) not in entries:
                starts += 1
        # with no dropped lines, a curve's chain breaks only at edge/corner events
        assert starts <= 1 + len(segs) // 4
