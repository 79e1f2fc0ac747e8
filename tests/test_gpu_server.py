"""Render server: continuous batching with admission by an HBM budget. Every
response equals the same request rendered alone (identical per-pixel code),
in a mix of sets, sizes and modes, under a squeezed budget and with several
batches in flight."""
import time

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
    for k, (n, grid) in enumerate(((300, 32), (1200, 64))):
        ls = synth.abc_lineset(n, 120, 60 + k, perturb=bool(k))
        out.append((grid, L.lineset_voxelize(ls.curve_off, grid, 32, xyz=ls.xyz, attr=ls.attr)))
    return out


def _requests(sets, n, seed):
    rng = np.random.default_rng(seed)
    luts = [U.dev(synth.lut_ramp(1.0)), U.dev(synth.lut_importance_alpha())]
    reqs = []
    for k in range(n):
        sid = int(rng.integers(0, len(sets)))
        grid = sets[sid][0]
        W, H = [(64, 64), (128, 72), (200, 150), (33, 17)][int(rng.integers(0, 4))]
        cam = synth.orbit_cameras((grid,) * 3, 1, 7000 + 100 * seed + k, W, H)[0]
        opaque = bool(rng.integers(0, 2))
        params = dict(radius=0.4, opaque=opaque, shading=1, mode=int(rng.integers(0, 4) == 0))
        reqs.append((sid, cam, luts[0] if opaque else luts[1], params))
    return reqs


def _alone(sets, req):
    sid, cam, lut, params = req
    return L.lineset_render(sets[sid][1], cam, lut, **params)


@pytest.mark.parametrize("budget_mb,slots,max_batch", [(4096, 2, 64), (8, 3, 4), (2, 1, 1)])
def test_responses_equal_alone(sets, budget_mb, slots, max_batch):
    resident = sum(s.info().device_bytes for _, s in sets)
    srv = L.Server(resident + budget_mb * (1 << 20), n_slots=slots, max_batch_views=max_batch)
    ids = [srv.add_lineset(s) for _, s in sets]
    reqs = _requests(sets, 40, budget_mb)
    outs, tickets = [], []
    for k, (sid, cam, lut, params) in enumerate(reqs):
        out = torch.full((cam.height, cam.width, 4), -1.0, device="cuda")
        outs.append(out)
        tickets.append(srv.submit(ids[sid], cam, lut, out, **params))
        if k % 7 == 3:
            time.sleep(0.002)                  # arrivals while batches run
    for t in tickets:
        assert srv.wait(t, timeout_us=30_000_000)
    st = srv.stats()
    print(f"[server budget={budget_mb}MB slots={slots} batch<={max_batch}] {st}", flush=True)
    assert st["completed"] == len(reqs) and st["queued"] == 0
    assert st["mean_batch"] <= max_batch
    for k, req in enumerate(reqs):
        ref = _alone(sets, req)
        torch.cuda.synchronize()
        assert torch.equal(outs[k], ref), f"request {k} differs from its standalone render"
    srv.close()


def test_admission_and_errors(sets):
    resident = sets[0][1].info().device_bytes
    # budget fits the set plus one 200x150 request at a time
    srv = L.Server(resident + 200 * 150 * 16 + 4096, n_slots=2, max_batch_views=8, max_queue=3)
    sid = srv.add_lineset(sets[0][1])
    grid = sets[0][0]
    lut = U.dev(synth.lut_ramp(1.0))
    big = synth.default_camera((grid,) * 3, 400, 400)
    with pytest.raises(L.LinesetError):      # larger than the budget can ever hold
        srv.submit(sid, big, lut, torch.empty((400, 400, 4), device="cuda"), radius=0.4)
    cam = synth.default_camera((grid,) * 3, 200, 150)
    outs = [torch.empty((150, 200, 4), device="cuda") for _ in range(12)]
    tickets, busy = [], 0
    for o in outs:
        try:
            tickets.append(srv.submit(sid, cam, lut, o, radius=0.4))
        except L.LinesetError as e:
            assert e.status == L.LS_EBUSY
            busy += 1
    for t in tickets:
        assert srv.wait(t, timeout_us=30_000_000)
    st = srv.stats()
    print(f"[admission] {st} busy={busy}", flush=True)
    assert st["completed"] == len(tickets) and st["mean_batch"] <= 1.0 + 1e-9
    assert 0 <= st["held_for_memory"] <= len(tickets)
    with pytest.raises(L.LinesetError):      # already collected
        srv.wait(tickets[0])
    srv.close()


def test_wait_timeout(sets):
    resident = sum(s.info().device_bytes for _, s in sets)
    srv = L.Server(resident + (64 << 20), n_slots=1, max_batch_views=1)
    sid = srv.add_lineset(sets[1][1])
    lut = U.dev(synth.lut_importance_alpha())
    cam = synth.default_camera((64,) * 3, 512, 512)
    outs = [torch.empty((512, 512, 4), device="cuda") for _ in range(60)]
    ts = [srv.submit(sid, cam, lut, o, radius=0.4, mode=1) for o in outs]
    # the last of 60 serialized requests cannot be done after zero wait
    assert srv.wait(ts[-1], timeout_us=0) is False
    for t in ts:
        assert srv.wait(t)
    srv.close()


def test_budget_rejects_resident_sets(sets):
    with pytest.raises(L.LinesetError):
        srv = L.Server(1024, n_slots=1)
        srv.add_lineset(sets[1][1])
