"""GPU parity: grid set-up, voxelization (CSR) and the density pyramid /
illumination grids against the oracle. Integer outputs are bit-exact."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1801_01155_amd as L
from paper_1801_01155_amd import synth
from tests import gpu_util as U
from tests.test_oracle_voxelize import _random_curves

pytestmark = pytest.mark.gpu


def _csr_equal(ls, ref, label):
    offs, recs = U.gpu_csr(ls)
    print(f"[csr {label}] records gpu={len(recs)} oracle={len(ref.records)}", flush=True)
    assert np.array_equal(offs, ref.offsets), f"{label}: offsets differ"
    assert np.array_equal(recs, ref.records), f"{label}: records differ"


def test_grid_setup_bit_exact():
    w, ls = U.workload("small")
    for grid in ((64, 64, 64), (37, 64, 20)):
        lat, lo_scale = L.lineset_grid_setup(U.dev(ls.xyz), grid)
        ref, lo, s = O.grid_setup(ls.xyz, grid)
        assert np.array_equal(lat.cpu().numpy(), ref)
        assert lo_scale[3] == s and list(lo_scale[:3]) == list(lo)


def test_voxelize_small_workload_from_xyz():
    w, ls = U.workload("small")
    ref, _ = U.oracle_csr_from_xyz(ls, w["grid"], w["bins"])
    s = L.lineset_voxelize(ls.curve_off, w["grid"], w["bins"], xyz=ls.xyz, attr=ls.attr)
    _csr_equal(s, ref, "small")
    info = s.info()
    cnt = np.diff(ref.offsets.astype(np.int64))
    assert info.nonempty_voxels == int((cnt > 0).sum()) and info.max_list == int(cnt.max())
    # the grid set-up made on the device during voxelization (bounds, scale)
    _, lo, sc = O.grid_setup(ls.xyz, (w["grid"],) * 3)
    assert list(info.lo_scale) == list(lo) + [sc]


def test_voxelize_xyz_degenerate_and_non_finite():
    # one vertex (zero extent: scale 0), and a non-finite coordinate (rejected)
    one = np.array([[0.25, -1.0, 3.0]], np.float32)
    s = L.lineset_voxelize(np.array([0, 1], np.int64), (8, 8, 8), 32, xyz=one)
    _, lo, sc = O.grid_setup(one, (8, 8, 8))
    assert s.info().n_records == 0 and list(s.info().lo_scale) == list(lo) + [sc]
    bad = np.array([[0.0, 0.0, 0.0], [1.0, np.nan, 0.0], [2.0, 1.0, 0.5]], np.float32)
    with pytest.raises(L.LinesetError):
        L.lineset_voxelize(np.array([0, 3], np.int64), (8, 8, 8), 32, xyz=bad)


@pytest.mark.parametrize("seed,step,bins", [(1, 64, 4), (2, 32, 32), (3, 1, 8), (4, 128, 64),
                                            (5, 16, 1), (6, 7, 16)])
def test_voxelize_edge_corner_cases(seed, step, bins):
    rng = np.random.default_rng(seed)
    grid = (5, 4, 6)
    lat, off = _random_curves(rng, 300, grid, step)
    attr = rng.integers(0, 256, len(off) - 1).astype(np.uint8)
    ref = O.voxelize(lat, off, attr, grid, bins)
    s = L.lineset_voxelize(off, grid, bins, lattice=lat, attr=attr)
    _csr_equal(s, ref, f"random seed={seed} step={step} bins={bins}")


def test_voxelize_medium_perturbed_and_deterministic():
    # 4000 x 200 perturbed streamlines on 96^3: many tiles, ragged tails
    ls = synth.abc_lineset(4000, 200, 12, perturb=True)
    ref, lat = U.oracle_csr_from_xyz(ls, 96, 32)
    a = L.lineset_voxelize(ls.curve_off, 96, 32, xyz=ls.xyz, attr=ls.attr)
    _csr_equal(a, ref, "medium xyz")
    b = L.lineset_voxelize(ls.curve_off, 96, 32, lattice=lat, attr=ls.attr)
    _csr_equal(b, ref, "medium lattice")


def test_voxelize_brick_counting_grid():
    # grids from 2^25 voxels count lines per voxel in brick-major (8^3) order;
    # sides that are not multiples of 8 leave partial bricks at the far faces
    grid = (517, 262, 251)
    assert grid[0] * grid[1] * grid[2] >= 1 << 25
    ls = synth.abc_lineset(3000, 200, 12, perturb=True)
    ref, lat = U.oracle_csr_from_xyz(ls, grid, 32)
    a = L.lineset_voxelize(ls.curve_off, grid, 32, xyz=ls.xyz, attr=ls.attr)
    _csr_equal(a, ref, "brick grid xyz")
    rng = np.random.default_rng(11)
    lat2, off2 = _random_curves(rng, 2000, grid, 16)
    b = L.lineset_voxelize(off2, grid, 8, lattice=lat2)
    _csr_equal(b, O.voxelize(lat2, off2, None, grid, 8), "brick grid random")
    info = b.info()
    cnt = np.diff(O.voxelize(lat2, off2, None, grid, 8).offsets.astype(np.int64))
    assert info.nonempty_voxels == int((cnt > 0).sum()) and info.max_list == int(cnt.max())


def test_voxelize_degenerate_inputs():
    # no curves, single-vertex curves, curves that never leave a voxel
    grid = (8, 8, 8)
    s = L.lineset_voxelize(np.array([0], np.int64), grid, 32, lattice=np.zeros((0, 3), np.int32))
    assert s.info().n_records == 0
    lat = np.array([[300, 300, 300], [310, 320, 330], [600, 600, 600]], np.int32)
    off = np.array([0, 1, 1, 3], np.int64)
    s = L.lineset_voxelize(off, grid, 32, lattice=lat)
    _csr_equal(s, O.voxelize(lat, off, None, grid, 32), "degenerate")


def test_voxelize_rejects_bad_input():
    lat = np.array([[0, 0, 0], [256 * 8, 0, 0]], np.int32)
    with pytest.raises(L.LinesetError):
        L.lineset_voxelize(np.array([0, 2]), (8, 8, 8), 32, lattice=lat)
    with pytest.raises(L.LinesetError):
        L.lineset_voxelize(np.array([0, 2]), (8, 8, 8), 24, lattice=lat[:1].repeat(2, 0))
    with pytest.raises(L.LinesetError):
        L.lineset_voxelize(np.array([1, 2]), (8, 8, 8), 32, lattice=lat[:1].repeat(2, 0))


# --- density pyramid and illumination grids ----------------------------------------
def _lod_case(grid=48, n=600):
    ls = synth.abc_lineset(n, 100, 21, perturb=True)
    ref, _ = U.oracle_csr_from_xyz(ls, grid, 32)
    s = L.lineset_voxelize(ls.curve_off, grid, 32, xyz=ls.xyz, attr=ls.attr)
    return ls, ref, s


# 48^3 and (37, 20, 29): every coarse level is small (built through LDS
# bricks, ragged odd sides); (130, 131, 129): its first coarse level (65 x 66
# x 65) has more than 2^18 voxels and gets a launch of its own, the rest go
# through bricks
@pytest.mark.parametrize("grid", [48, (37, 20, 29), (130, 131, 129)])
def test_lod_pyramid_parity(grid):
    ls, ref, s = _lod_case(grid=grid)
    lut = synth.lut_importance_alpha()
    L.lineset_build_lod(s, U.dev(lut), opaque=False)
    torch.cuda.synchronize()
    cnt, ln, rho, dims, loff = O.lod(ref, grid, 32, lut, opaque=False)
    for what, r in ((L.EXPORT_LOD_COUNT, cnt), (L.EXPORT_LOD_LEN, ln), (L.EXPORT_LOD_RHO, rho)):
        g = L.lineset_export(s, what).cpu().numpy().astype(np.float64)
        err = np.abs(g - r) / np.maximum(np.abs(r), 1e-30)
        print(f"[lod grid={grid} field={what}] max_rel_err={err.max():.3e}", flush=True)
        assert np.allclose(g, r, rtol=1e-5, atol=1e-12)
    assert s.info().n_levels == len(dims)


@pytest.mark.parametrize("grid,aperture,radius,separate",
                         [(40, 1.0, 15.0, False), ((37, 20, 29), 1.0, 15.0, False),
                          (40, 0.5, 15.0, False), ((37, 20, 29), 1.0, 6.0, False),
                          (40, 1.0, 15.0, True)])
def test_illumination_grids_parity(grid, aperture, radius, separate):
    # Cubic and ragged grids (partial tiles). Aperture 1, radius 15: the
    # column kernel specialised for levels 0..3, shadow fused; radius 6: the
    # generic column kernel (3 samples per cone), shadow fused; aperture 0.5
    # puts several samples on one level and boxes beyond the LDS budget
    # (per-voxel kernels). separate: AO and shadow built by two calls (the
    # column kernel alone, then the per-voxel shadow kernel).
    ls, ref, s = _lod_case(grid=grid, n=800)
    lut = synth.lut_importance_alpha()
    light = synth.LIGHT_DIR
    if separate:
        L.lineset_build_lod(s, U.dev(lut), opaque=False, build_ao=True, ao_cones=16,
                            ao_radius=radius, cone_aperture=aperture)
        L.lineset_build_lod(s, U.dev(lut), opaque=False, cone_aperture=aperture,
                            build_shadow=True, light_dir=light)
    else:
        L.lineset_build_lod(s, U.dev(lut), opaque=False, build_ao=True, ao_cones=16,
                            ao_radius=radius, cone_aperture=aperture, build_shadow=True,
                            light_dir=light)
    torch.cuda.synchronize()
    _, _, rho, _, _ = O.lod(ref, grid, 32, lut, opaque=False)
    ao = O.ao_grid(rho, grid, 16, radius, aperture)
    sh = O.shadow_grid(rho, grid, np.array(light, dtype=np.float32).astype(np.float64), aperture)
    gao = L.lineset_export(s, L.EXPORT_AO).cpu().numpy()
    gsh = L.lineset_export(s, L.EXPORT_SHADOW).cpu().numpy()
    print(f"[illum grid={grid} aperture={aperture} radius={radius} separate={separate}] "
          f"ao max_abs_err={np.abs(gao - ao).max():.3e} "
          f"sh max_abs_err={np.abs(gsh - sh).max():.3e} ao_min={ao.min():.3f} sh_min={sh.min():.3f}",
          flush=True)
    assert ao.min() < 0.95 and sh.min() < 0.95
    assert np.abs(gao - ao).max() < 1e-5
    assert np.abs(gsh - sh).max() < 1e-5


def test_memory_cache_reuse_and_trim():
    """Set buffers and voxelizer temporaries come from the device memory
    cache: a destroyed set's blocks are reused (stale contents must not leak
    into the next CSR) and trimming returns them."""
    dev = torch.cuda.current_device()
    ls = synth.abc_lineset(4000, 200, 12, perturb=True)
    ref, _ = U.oracle_csr_from_xyz(ls, 96, 32)
    other = synth.abc_lineset(3000, 150, 13, perturb=True)
    ref2, _ = U.oracle_csr_from_xyz(other, 96, 32)
    a = L.lineset_voxelize(ls.curve_off, 96, 32, xyz=ls.xyz, attr=ls.attr)
    _csr_equal(a, ref, "cache first")
    a.close()
    st = L.lineset_pool_stats(dev)
    assert st["cached_bytes"] > 0 and st["held_bytes"] >= st["cached_bytes"]
    b = L.lineset_voxelize(other.curve_off, 96, 32, xyz=other.xyz, attr=other.attr)
    _csr_equal(b, ref2, "cache reused by another set")
    b.close()
    held = L.lineset_pool_stats(dev)["held_bytes"]
    c = L.lineset_voxelize(ls.curve_off, 96, 32, xyz=ls.xyz, attr=ls.attr)
    _csr_equal(c, ref, "cache reused by the same shape")
    assert L.lineset_pool_stats(dev)["held_bytes"] == held    # no new device memory
    c.close()
    L.lineset_pool_trim()
    st = L.lineset_pool_stats(dev)
    print(f"[pool] after trim {st}", flush=True)
    assert st["cached_bytes"] == 0
    with pytest.raises(L.LinesetError):
        L.lineset_pool_stats(-1)
