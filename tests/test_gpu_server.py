"""Render server: continuous batching with admission by memory. Every
response equals the same request rendered alone (identical per-pixel code),
in a mix of sets, sizes, modes and shadings (AO/shadow included), under a
squeezed budget and with several batches in flight; a seeded subset of the
responses is also checked against the oracle, fed the oracle's own CSR and
illumination grids. The output arena's admission holds requests until
blocks are collected."""
import time

import numpy as np
import pytest
import torch

import oracle as O
import paper_1801_01155_amd as L
from paper_1801_01155_amd import synth
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

LIGHT = synth.LIGHT_DIR


@pytest.fixture(scope="module")
def sets():
    """Two sets with density pyramids, AO and shadow grids (GPU and oracle)."""
    out = []
    lut = synth.lut_importance_alpha()
    for k, (n, grid) in enumerate(((300, 32), (1200, 64))):
        ls = synth.abc_lineset(n, 120, 60 + k, perturb=bool(k))
        s = L.lineset_voxelize(ls.curve_off, grid, 32, xyz=ls.xyz, attr=ls.attr)
        L.lineset_build_lod(s, U.dev(lut), opaque=False, build_ao=True, build_shadow=True,
                            light_dir=LIGHT)
        ref, _ = U.oracle_csr_from_xyz(ls, grid, 32)
        _, _, rho, _, _ = O.lod(ref, grid, 32, lut, opaque=False)
        ao = O.ao_grid(rho, grid, 16, 15.0, 1.0)
        sh = O.shadow_grid(rho, grid, np.array(LIGHT, np.float32).astype(np.float64))
        out.append(dict(grid=grid, set=s, csr=ref, ao=ao, sh=sh))
    torch.cuda.synchronize()
    return out


def _requests(sets, n, seed):
    """Requests over sets, sizes, opaque/transparent, modes 0/1 and shadings 1/2."""
    rng = np.random.default_rng(seed)
    luts = [synth.lut_ramp(1.0), synth.lut_importance_alpha()]
    dluts = [U.dev(x) for x in luts]
    reqs = []
    for k in range(n):
        sid = int(rng.integers(0, len(sets)))
        grid = sets[sid]["grid"]
        W, H = [(64, 64), (128, 72), (200, 150), (33, 17)][int(rng.integers(0, 4))]
        cam = synth.orbit_cameras((grid,) * 3, 1, 7000 + 100 * seed + k, W, H)[0]
        opaque = bool(rng.integers(0, 2))
        params = dict(radius=0.4, opaque=opaque, shading=int(rng.integers(1, 3)),
                      mode=int(rng.integers(0, 4) == 0), light_dir=LIGHT)
        reqs.append((sid, cam, dluts[0] if opaque else dluts[1], luts[0] if opaque else luts[1],
                     params))
    return reqs


def _alone(sets, req):
    sid, cam, lut, _, params = req
    return L.lineset_render(sets[sid]["set"], cam, lut, **params)


def _oracle(sets, req):
    sid, cam, _, lut_np, params = req
    S = sets[sid]
    img, _ = O.render(S["csr"], S["grid"], 32, cam, ao=S["ao"], sh=S["sh"], lut=lut_np,
                      **params)
    return img


@pytest.mark.parametrize("budget_mb,slots,max_batch", [(4096, 2, 64), (8, 3, 4), (2, 1, 1)])
def test_responses_equal_alone_and_oracle(sets, budget_mb, slots, max_batch):
    resident = sum(S["set"].info().device_bytes for S in sets)
    srv = L.Server(resident + budget_mb * (1 << 20), n_slots=slots, max_batch_views=max_batch)
    ids = [srv.add_lineset(S["set"]) for S in sets]
    reqs = _requests(sets, 40, budget_mb)
    assert {r[4]["shading"] for r in reqs} == {1, 2}
    outs, tickets = [], []
    for k, (sid, cam, lut, _, params) in enumerate(reqs):
        # the fill is queued on the current stream; the server orders the render after it
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
    # a seeded subset against the oracle, covering both shadings and both modes
    rng = np.random.default_rng(100 + budget_mb)
    picks = set(rng.choice(len(reqs), 8, replace=False).tolist())
    for sh in (1, 2):
        picks.add(next(k for k, r in enumerate(reqs) if r[4]["shading"] == sh))
    picks.add(next(k for k, r in enumerate(reqs) if r[4]["mode"] == 1))
    for k in sorted(picks):
        p = reqs[k][4]
        U.assert_image_parity(outs[k].cpu().numpy(), _oracle(sets, reqs[k]),
                              f"served request {k} (shading {p['shading']}, mode {p['mode']}, "
                              f"opaque {p['opaque']}) vs oracle")
    srv.close()


def test_output_arena_admission(sets):
    """Arena of two 200x150 images: at most two such requests hold blocks at
    once; the rest wait at the head until results are collected. Images equal
    the standalone renders."""
    W, H = 200, 150
    block = W * H * 16
    resident = sets[1]["set"].info().device_bytes
    srv = L.Server(resident + 2 * block + 4096, n_slots=2, max_batch_views=8,
                   output_arena_bytes=2 * block)
    sid = srv.add_lineset(sets[1]["set"])
    grid = sets[1]["grid"]
    lut = U.dev(synth.lut_importance_alpha())
    cams = synth.orbit_cameras((grid,) * 3, 6, 77, W, H)
    params = dict(radius=0.4, opaque=False, shading=2, light_dir=LIGHT)
    tickets = [srv.submit(sid, c, lut, None, **params) for c in cams]
    time.sleep(0.05)
    st = srv.stats()
    print(f"[arena] while waiting: {st}", flush=True)
    assert st["arena_in_use"] <= 2 * block
    for c, t in zip(cams, tickets):
        assert srv.wait(t, timeout_us=30_000_000)
        got = srv.result(t, torch.empty((H, W, 4), device="cuda"))
        ref = L.lineset_render(sets[1]["set"], c, lut, **params)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
    st = srv.stats()
    print(f"[arena] done: {st}", flush=True)
    assert st["completed"] == len(cams) and st["arena_in_use"] == 0
    assert st["held_for_memory"] >= 1
    with pytest.raises(L.LinesetError):      # already collected
        srv.result(tickets[0], torch.empty((H, W, 4), device="cuda"))
    with pytest.raises(L.LinesetError):      # larger than the arena
        srv.submit(sid, synth.default_camera((grid,) * 3, 400, 400), lut, None, **params)
    srv.close()


def test_grids_built_after_adding_count_against_budget():
    ls = synth.abc_lineset(200, 60, 99)
    s = L.lineset_voxelize(ls.curve_off, 32, 32, xyz=ls.xyz, attr=ls.attr)
    srv = L.Server(s.info().device_bytes + (64 << 20), n_slots=1)
    srv.add_lineset(s)
    before = srv.stats()["resident_bytes"]
    L.lineset_build_lod(s, U.dev(synth.lut_importance_alpha()), build_ao=True,
                        build_shadow=True, light_dir=LIGHT)
    cam = synth.default_camera((32,) * 3, 16, 16)
    t = srv.submit(0, cam, U.dev(synth.lut_ramp(1.0)), torch.empty((16, 16, 4), device="cuda"),
                   radius=0.4, shading=2, light_dir=LIGHT)
    assert srv.wait(t, timeout_us=30_000_000)
    after = srv.stats()["resident_bytes"]
    print(f"[resident] {before} -> {after}", flush=True)
    assert after > before
    srv.close()


def test_admission_and_errors(sets):
    resident = sets[0]["set"].info().device_bytes
    # budget fits the set plus one 200x150 request at a time
    srv = L.Server(resident + 200 * 150 * 16 + 4096, n_slots=2, max_batch_views=8, max_queue=3)
    sid = srv.add_lineset(sets[0]["set"])
    grid = sets[0]["grid"]
    lut = U.dev(synth.lut_ramp(1.0))
    big = synth.default_camera((grid,) * 3, 400, 400)
    with pytest.raises(L.LinesetError):      # larger than the budget can ever hold
        srv.submit(sid, big, lut, torch.empty((400, 400, 4), device="cuda"), radius=0.4)
    with pytest.raises(L.LinesetError):      # no output and no arena
        srv.submit(sid, big, lut, None, radius=0.4)
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
    resident = sum(S["set"].info().device_bytes for S in sets)
    srv = L.Server(resident + (64 << 20), n_slots=1, max_batch_views=1)
    sid = srv.add_lineset(sets[1]["set"])
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
        srv.add_lineset(sets[1]["set"])
