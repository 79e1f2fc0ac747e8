"""GPU parity of per-vertex attributes (section "Curve voxelization": line
attributes interpolated to the line-face intersection points) against the
oracle: records and per-line endpoint attributes bit-exact, the density
pyramid (from the records' mean attribute) to relative 1e-5, and images
whose colour and opacity come from the attribute interpolated along each
line, at the usual bar, in both candidate modes; the batched and served
paths equal the plain renderer."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1801_01155_amd as L
from paper_1801_01155_amd import synth
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _vertex_attr(ls, seed):
    """A smooth attribute along each curve: a ramp between two random
    levels plus a wiggle, one byte per vertex."""
    rng = np.random.default_rng(seed)
    va = np.empty(ls.xyz.shape[0], np.uint8)
    for c in range(ls.n_curves):
        v0, v1 = int(ls.curve_off[c]), int(ls.curve_off[c + 1])
        n = v1 - v0
        a, b = rng.integers(0, 256, 2)
        s = np.linspace(0.0, 1.0, n)
        val = a + (b - a) * s + 30.0 * np.sin(9.0 * s + c)
        va[v0:v1] = np.clip(np.rint(val), 0, 255).astype(np.uint8)
    return va


@pytest.fixture(scope="module")
def attr_set():
    ls = synth.abc_lineset(2000, 150, 13, perturb=True)
    va = _vertex_attr(ls, 1)
    grid, bins = 72, 32
    lat, _, _ = O.grid_setup(ls.xyz, grid)
    ref = O.voxelize(lat, ls.curve_off, ls.attr, grid, bins, vattr=va)
    s = L.lineset_voxelize(ls.curve_off, grid, bins, xyz=ls.xyz, attr=ls.attr, vattr=va)
    return dict(ls=ls, va=va, lat=lat, grid=grid, bins=bins, ref=ref, s=s)


def test_records_and_endpoint_attributes_bit_exact(attr_set):
    A = attr_set
    offs, recs = U.gpu_csr(A["s"])
    ends = L.lineset_export(A["s"], L.EXPORT_ENDS).cpu().numpy().view(np.uint16)
    print(f"[attributes] records={len(recs)}", flush=True)
    assert np.array_equal(offs, A["ref"].offsets)
    assert np.array_equal(recs, A["ref"].records)
    assert np.array_equal(ends, A["ref"].ends)
    assert L.lineset_info(A["s"]).has_vertex_attr == 1
    # lattice input, odd grid and bins
    grid = (41, 30, 27)
    lat, _, _ = O.grid_setup(A["ls"].xyz, grid)
    ref = O.voxelize(lat, A["ls"].curve_off, None, grid, 8, vattr=A["va"])
    s = L.lineset_voxelize(A["ls"].curve_off, grid, 8, lattice=lat, vattr=A["va"])
    o2, r2 = U.gpu_csr(s)
    e2 = L.lineset_export(s, L.EXPORT_ENDS).cpu().numpy().view(np.uint16)
    assert np.array_equal(o2, ref.offsets) and np.array_equal(r2, ref.records)
    assert np.array_equal(e2, ref.ends)


def test_endpoint_attributes_on_brick_counting_grid(attr_set):
    # grids from 2^25 voxels count lines in brick-major order (ragged bricks
    # at the far faces); the attribute instance of the emit pass takes the
    # same path
    A = attr_set
    grid = (517, 262, 251)
    lat, _, _ = O.grid_setup(A["ls"].xyz, grid)
    ref = O.voxelize(lat, A["ls"].curve_off, A["ls"].attr, grid, 32, vattr=A["va"])
    s = L.lineset_voxelize(A["ls"].curve_off, grid, 32, xyz=A["ls"].xyz, attr=A["ls"].attr,
                           vattr=A["va"])
    offs, recs = U.gpu_csr(s)
    ends = L.lineset_export(s, L.EXPORT_ENDS).cpu().numpy().view(np.uint16)
    print(f"[attributes brick grid] records={len(recs)}", flush=True)
    assert np.array_equal(offs, ref.offsets) and np.array_equal(recs, ref.records)
    assert np.array_equal(ends, ref.ends)


def test_density_from_mean_attribute(attr_set):
    A = attr_set
    lut = synth.lut_importance_alpha()
    L.lineset_build_lod(A["s"], U.dev(lut), opaque=False)
    _, _, rho, _, _ = O.lod(A["ref"], A["grid"], A["bins"], lut, opaque=False)
    g = L.lineset_export(A["s"], L.EXPORT_LOD_RHO).cpu().numpy().astype(np.float64)
    assert np.allclose(g, rho, rtol=1e-5, atol=1e-12)


@pytest.mark.parametrize("mode,opaque,shading,dist", [(0, True, 1, False), (0, False, 0, False),
                                                      (0, False, 1, True), (1, False, 1, False),
                                                      (1, True, 0, False)])
def test_render_with_interpolated_attributes(attr_set, mode, opaque, shading, dist):
    A = attr_set
    lut = synth.lut_importance_alpha(0.05, 0.8)
    cam = synth.orbit_cameras((A["grid"],) * 3, 1, 31 + mode, 160, 120)[0]
    params = dict(mode=mode, radius=0.4, opaque=opaque, shading=shading, distance_alpha=dist,
                  alpha_stop=0.95, merge_curves=True)
    g = L.lineset_render(A["s"], cam, U.dev(lut), **params)
    torch.cuda.synchronize()
    r, _ = O.render(A["ref"], A["grid"], A["bins"], cam, lut=lut, **params)
    assert r[..., 3].mean() > 0.02
    U.assert_image_parity(g.cpu().numpy(), r,
                          f"attributes mode={mode} opaque={opaque} shading={shading} dist={dist}")
    # the interpolation shows: the same lines with the records' mean attribute differ
    plain = O.OracleCsr(A["ref"].offsets, A["ref"].records, 0, 0)
    r2, _ = O.render(plain, A["grid"], A["bins"], cam, lut=lut, **params)
    assert np.abs(r2 - r).max() > 1e-2


def test_batch_and_server_equal_alone(attr_set):
    A = attr_set
    lut = U.dev(synth.lut_importance_alpha())
    items = []
    for k in range(4):
        cam = synth.orbit_cameras((A["grid"],) * 3, 1, 90 + k, 48 + 8 * k, 40)[0]
        p = dict(radius=0.4, opaque=k % 2 == 0, shading=1, mode=int(k == 3))
        items.append((A["s"], cam, lut, torch.full((40, 48 + 8 * k, 4), -1.0, device="cuda"), p))
    b = L.Batch(items)
    b.render()
    torch.cuda.synchronize()
    alone = [L.lineset_render(s, cam, lt, **p) for (s, cam, lt, _, p) in items]
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        assert torch.equal(it[3], alone[k]), f"batched view {k}"
    b.close()
    srv = L.Server(1 << 34, n_slots=2, max_batch_views=8)
    sid = srv.add_lineset(A["s"])
    outs = [torch.full_like(it[3], -1.0) for it in items]
    tickets = [srv.submit(sid, it[1], it[2], out=o, **it[4]) for it, o in zip(items, outs)]
    for t in tickets:
        srv.wait(t)
    torch.cuda.synchronize()
    for k in range(len(items)):
        assert torch.equal(outs[k], alone[k]), f"served view {k}"
    srv.close()


def test_update_rejects_attribute_sets(attr_set):
    with pytest.raises(L.LinesetError) as e:
        L.lineset_update(attr_set["s"], remove=torch.tensor([0], dtype=torch.int64))
    assert e.value.status == L.LS_EUNSUPPORTED
