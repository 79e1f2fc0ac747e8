"""The allocation-free batch entry point (lineset_render_batch_static) gives
the same images as the allocating one-shot batch (lineset_render_batch), on
two calls in a row (the second with fewer, smaller views, so stale
descriptors or queue counters left in the fixed scratch would show), and
rejects batches beyond its fixed capacity."""
import numpy as np
import pytest
import torch

import paper_1801_01155_amd as L
from paper_1801_01155_amd import synth
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sets():
    out = []
    for k, (n, grid) in enumerate(((400, 32), (1500, 64))):
        ls = synth.abc_lineset(n, 120, 60 + k, perturb=bool(k % 2))
        out.append((grid, L.lineset_voxelize(ls.curve_off, grid, 32, xyz=ls.xyz, attr=ls.attr)))
    return out


def _items(sets, n_views, max_side, seed):
    rng = np.random.default_rng(seed)
    luts = [U.dev(synth.lut_ramp(1.0)), U.dev(synth.lut_importance_alpha())]
    items = []
    for v in range(n_views):
        grid, s = sets[v % len(sets)]
        W = int(rng.integers(9, max_side))
        H = int(rng.integers(9, max_side))
        cam = synth.orbit_cameras((grid,) * 3, 1, 500 * seed + v, W, H,
                                  orthographic=bool(rng.integers(0, 2)))[0]
        opaque = v % 2 == 0
        params = dict(radius=0.4, opaque=opaque, mode=int(v % 3 == 2), shading=int(v % 2),
                      merge_curves=True, alpha_stop=0.95)
        items.append((s, cam, luts[0] if opaque else luts[1],
                      torch.full((H, W, 4), -1.0, device="cuda"), params))
    return items


def _check_against_one_shot(items, label):
    L.lineset_render_batch_static(items)
    got = [it[3].clone() for it in items]
    for it in items:
        it[3].fill_(-2.0)
    L.lineset_render_batch(items)
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        assert torch.equal(got[k], it[3]), f"{label}: view {k} differs from lineset_render_batch"
        assert bool((got[k][..., 3] >= 0).all()), f"{label}: view {k} left unwritten pixels"
    print(f"[no-alloc] {label}: {len(items)} views equal", flush=True)


def test_static_batch_equals_one_shot_twice(sets):
    big = _items(sets, 12, 260, 1)
    _check_against_one_shot(big, "first call, 12 views")
    small = _items(sets, 3, 40, 2)
    _check_against_one_shot(small, "second call, 3 smaller views")


def test_static_batch_rejects_too_many_views(sets):
    items = _items(sets, 1, 16, 3) * 257
    with pytest.raises(L.LinesetError) as e:
        L.lineset_render_batch_static(items)
    assert e.value.status == -1
