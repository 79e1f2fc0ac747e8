"""Batched persistent rendering: every view of a mixed batch (several sets,
uneven sizes, opaque/transparent, both modes) equals the same view rendered
alone (identical per-pixel code path); autotuned and graph-replayed batches
too. One view per batch is also checked against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1801_01155_amd as L
from paper_1801_01155_amd import synth
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sets():
    out = []
    for k, (n, grid) in enumerate(((400, 32), (1500, 64), (3000, 96))):
        ls = synth.abc_lineset(n, 120, 40 + k, perturb=bool(k % 2))
        s = L.lineset_voxelize(ls.curve_off, grid, 32, xyz=ls.xyz, attr=ls.attr)
        out.append((ls, grid, s))
    return out


def _items(sets, n_views, seed):
    rng = np.random.default_rng(seed)
    luts = [U.dev(synth.lut_ramp(1.0)), U.dev(synth.lut_importance_alpha())]
    items = []
    for v in range(n_views):
        ls, grid, s = sets[v % len(sets)]
        W = int(rng.integers(17, 300))
        H = int(rng.integers(9, 200))
        cam = synth.orbit_cameras((grid,) * 3, 1, 1000 * seed + v, W, H,
                                  orthographic=bool(rng.integers(0, 2)))[0]
        opaque = bool(v % 2 == 0)
        params = dict(radius=0.4, opaque=opaque, mode=int(v % 5 == 4), shading=int(v % 3 != 0),
                      merge_curves=True, alpha_stop=0.95, distance_alpha=v % 4 == 1)
        out = torch.full((H, W, 4), -1.0, device="cuda")
        items.append((s, cam, luts[0] if opaque else luts[1], out, params))
    return items


def _alone(item):
    s, cam, lut, _, params = item
    return L.lineset_render(s, cam, lut, **params)


@pytest.mark.parametrize("autotune,graph", [(False, False), (True, False), (True, True)])
def test_batch_equals_alone(sets, autotune, graph):
    items = _items(sets, 24, 1 + int(autotune) + 2 * int(graph))
    b = L.Batch(items, autotune=autotune, graph=graph)
    for it in items:
        it[3].fill_(-1.0)
    b.render()
    torch.cuda.synchronize()
    print(f"[batch] config={b.config()}", flush=True)
    for k, it in enumerate(items):
        ref = _alone(it)
        torch.cuda.synchronize()
        assert torch.equal(it[3], ref), f"view {k} differs from its standalone render"
    # replays give the same images
    for it in items:
        it[3].fill_(-1.0)
    b.render()
    b.render()
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        assert torch.equal(it[3], _alone(it)), f"view {k} differs on replay"
    b.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_repeated_launches_equal_alone(sets, graph):
    """Every launch of a batch (eager or graph replay) gives each view's
    image: outputs cleared to NaN before each of four launches, so that a
    tile left out would show."""
    items = _items(sets, 24, 11 + int(graph))
    b = L.Batch(items, autotune=False, graph=graph)
    print(f"[batch] config={b.config()}", flush=True)
    refs = [_alone(it).clone() for it in items]
    torch.cuda.synchronize()
    for rep in range(4):
        for it in items:
            it[3].fill_(float("nan"))
        b.render()
        torch.cuda.synchronize()
        for k, (it, ref) in enumerate(zip(items, refs)):
            assert torch.equal(it[3], ref), f"launch {rep + 1} view {k}"
    b.close()


def test_batch_view_matches_oracle(sets):
    ls, grid, s = sets[1]
    ref, _ = U.oracle_csr_from_xyz(ls, grid, 32)
    lut = synth.lut_importance_alpha()
    cam = synth.default_camera((grid,) * 3, 160, 90)
    out = torch.empty((90, 160, 4), device="cuda")
    other = torch.empty((40, 33, 4), device="cuda")
    params = dict(radius=0.4, opaque=False, shading=1)
    items = [(s, cam, U.dev(lut), out, params),
             (sets[0][2], synth.default_camera((32,) * 3, 33, 40), U.dev(lut), other, params)]
    L.lineset_render_batch(items)
    r, _ = O.render(ref, grid, 32, cam, lut=lut, **params)
    U.assert_image_parity(out.cpu().numpy(), r, "batched view vs oracle")


def test_batch_counters_match_sum_of_views(sets):
    items = _items(sets, 6, 9)
    b = L.Batch(items)
    kb = b.render_counted()
    tot = {}
    for it in items:
        s, cam, lut, out, params = it
        _, k = L.lineset_render_counted(s, cam, lut, out=out, **params)
        for n, v in k.items():
            tot[n] = tot.get(n, 0) + v
    print(f"[batch counters] batch={kb} views={tot}", flush=True)
    for n in ("visited", "nonempty", "tested", "hits", "fragments"):
        assert kb[n] == tot[n]


def test_batch_rejects_invalid_view(sets):
    items = _items(sets, 3, 5)
    bad = list(items[1])
    bad[4] = dict(bad[4], radius=-1.0)
    with pytest.raises(L.LinesetError):
        L.Batch([items[0], tuple(bad), items[2]])


def test_every_autotuner_plan_equals_alone(sets):
    """Each plan the autotuner can pick (tile shape x grid size) renders the
    batch's views exactly as the plain renderer does."""
    plans = L.batch_candidates()
    assert len(plans) == 12 and len(set(plans)) == 12
    items = _items(sets, 14, 9)
    alone = [_alone(it) for it in items]
    torch.cuda.synchronize()
    for plan in plans:
        for it in items:
            it[3].fill_(-1.0)
        b = L.Batch(items, plan=plan)
        cfg = b.config()
        assert (cfg["waves_x"], cfg["waves_y"]) == plan[:2] and cfg["autotuned"] == 0
        b.render()
        torch.cuda.synchronize()
        for k, it in enumerate(items):
            assert torch.equal(it[3], alone[k]), f"plan {plan}: view {k} differs"
        b.close()
    with pytest.raises(L.LinesetError):
        L.Batch(items, plan=(3, 3, 1))
    with pytest.raises(L.LinesetError):
        L.Batch(items, plan=(2, 2, 0))
