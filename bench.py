"""Benchmark: the whole voxel ray-casting path on one MI355X.

One step = one pass of the hot path over the "scale" workload (100k ABC-flow
streamlines x 200 vertices, perturbed; 256^3 grid, 32^2 bins; transparent
lines, alpha in [0.02, 0.5]; 1920x1080 perspective):
    voxelize (grid set-up, clipping, quantization, CSR) -> density pyramid ->
    AO + soft-shadow grids -> render one frame (AO/shadow shading).
Inputs (float vertices, curve offsets, attributes, LUT) are resident in HBM
before timing starts. Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_CAL_BYTES = 2 << 30

# HBM bytes the ray caster moves per launch on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) of
#   python3 bench.py --steps 2 --warmup 1 --no-batch --no-serve --no-cpu-baseline
#       --no-gi --no-vdi --no-update --copy-calibration
# (the two timed steps' dispatches), each scaled by the counter's reading for
# the appended 2 GiB copy (true bytes / counted bytes). The figure holds for
# the kernel source it was measured on only: bench reports it when
# csrc/render.hip still has this sha256, else null.
RENDER_TRAFFIC = {
    "render_hip_sha256": "57708021c185b83ec7d01373ce499af607c3c09f6ba1bff7b17d4d6f946dd193",
    "bytes_per_launch": 122445904,
}
# Counters of the same launch and source, from one rocprofv3 --pmc run
# (SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_ACTIVE_INST_VALU
# SQ_THREAD_CYCLES_VALU TCC_HIT_sum TCC_MISS_sum): L2 hit = hits / (hits +
# misses); VALU lane use = thread-cycles / (64 x wave instructions); waits =
# SQ_WAIT_ANY / SQ_WAVE_CYCLES.
RENDER_COUNTERS = {"l2_hit": 0.822, "valu_lane_use": 0.341, "wait_frac": 0.350}
# fp32 operations of one ray-capsule test (two sphere quadratics, the
# projected cylinder quadratic and its slab clip), counted from the kernel
# source; the VALU figure of the roofline is tests x this / launch time.
CAPSULE_FLOPS = 100
VALU_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="scale")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched / served comparison")
    ap.add_argument("--cpu-sample-rows", type=int, default=8,
                    help="oracle renders every k-th image row")
    ap.add_argument("--no-update", action="store_true",
                    help="skip the incremental-update leg")
    ap.add_argument("--no-gi", action="store_true",
                    help="skip the global-illumination (512^3) leg")
    ap.add_argument("--no-vdi", action="store_true",
                    help="skip the view-dependent illumination leg")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the open-loop serving sweep")
    ap.add_argument("--serve-rates", default="10,25,50,100,200,500,1000,2000,4000",
                    help="Poisson arrival rates (requests/s)")
    ap.add_argument("--serve-seconds", type=float, default=4.0,
                    help="arrivals per rate: max(100, rate * seconds), capped")
    ap.add_argument("--serve-max-requests", type=int, default=2000)
    ap.add_argument("--serve-arena-mib", type=float, default=128.0,
                    help="server-owned output arena (HBM budget beyond the resident sets)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="append one 2 GiB device-to-device copy (the reference kernel "
                         "that scales rocprofv3 FETCH_SIZE / WRITE_SIZE readings)")
    return ap.parse_args()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_1thread(w, cam, lut, light, csr, rho, t_vox):
    """The same step on one host thread: the voxelizer (single-threaded, timed
    in full by the caller) and the pyramid in full, AO + shadow for 4
    z-planes of voxels, render every 64th row; samples scaled to the step."""
    import oracle as O
    grid, bins = w["grid"], w["bins"]
    t = time.perf_counter()
    O.lod(csr, grid, bins, lut, opaque=w["opaque"])
    t_lod = time.perf_counter() - t
    G2 = grid * grid
    v0, v1 = (grid // 2) * G2, (grid // 2 + 4) * G2
    L64 = np.array(light, np.float32).astype(np.float64)
    t = time.perf_counter()
    O.ao_grid_part(rho, grid, v0, v1, 16, 15.0, 1.0, threads=1)
    O.shadow_grid_part(rho, grid, L64, v0, v1, threads=1)
    t_illum = t_lod + (time.perf_counter() - t) * (grid ** 3 / (v1 - v0))
    W, H = cam.width, cam.height
    rows = np.arange(0, H, 64)
    pix = (rows[:, None] * W + np.arange(W)[None, :]).ravel()
    ao = np.full(grid ** 3, 0.5)
    sh = np.full(grid ** 3, 0.5)
    t = time.perf_counter()
    O.render(csr, grid, bins, cam, pixels=pix, ao=ao, sh=sh, threads=1, lut=lut,
             radius=w["radius"], opaque=w["opaque"], shading=2, light_dir=light)
    t_render = (time.perf_counter() - t) * (W * H / len(pix))
    step = t_vox + t_illum + t_render
    return {"value": W * H / step / 1e6, "unit": "Mrays/s", "cores": 1,
            "sample": (f"voxelize in full; LoD full; AO+shadow for {v1 - v0} voxels "
                       f"(x{grid ** 3 / (v1 - v0):.0f}); render {len(pix)} pixels (every 64th "
                       f"row); per-step s: vox {t_vox:.2f} illum {t_illum:.2f} "
                       f"render {t_render:.2f}")}


def cpu_baseline(ls, w, cam, lut, light, row_stride):
    """The oracle, untuned, on the host cores: grid set-up and voxelization in
    full (single-threaded code), LoD + AO + shadow grids in full, render every
    row_stride-th row (scaled to the frame). Also the same step on one thread
    (smaller AO/shadow and render samples)."""
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    grid, bins = w["grid"], w["bins"]
    t = time.perf_counter()
    lat, _, _ = O.grid_setup(ls.xyz, grid)
    csr = O.voxelize(lat, ls.curve_off, ls.attr, grid, bins)
    t_vox = time.perf_counter() - t
    del lat
    t = time.perf_counter()
    _, _, rho, _, _ = O.lod(csr, grid, bins, lut, opaque=w["opaque"])
    ao = O.ao_grid(rho, grid, 16, 15.0, 1.0, threads=threads)
    sh = O.shadow_grid(rho, grid, np.array(light, np.float32).astype(np.float64), threads=threads)
    t_illum = time.perf_counter() - t
    W, H = cam.width, cam.height
    rows = np.arange(0, H, row_stride)
    pix = (rows[:, None] * W + np.arange(W)[None, :]).ravel()
    t = time.perf_counter()
    O.render(csr, grid, bins, cam, pixels=pix, ao=ao, sh=sh, threads=threads, lut=lut,
             radius=w["radius"], opaque=w["opaque"], shading=2, light_dir=light)
    t_render = (time.perf_counter() - t) * (W * H / len(pix))
    step = t_vox + t_illum + t_render
    one = cpu_baseline_1thread(w, cam, lut, light, csr, rho, t_vox)
    return {
        "value": W * H / step / 1e6,
        "unit": "Mrays/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": _cpu_model(),
        "one_thread": one,
        "sample": (f"grid set-up + voxelize all {ls.n_curves} curves; "
                   f"LoD+AO+shadow grids full; render {len(pix)} of {W * H} pixels "
                   f"(every {row_stride}th row); per-step s: vox {t_vox:.2f} "
                   f"illum {t_illum:.2f} render {t_render:.2f}"),
    }


def batched_vs_plain(L, synth, torch, dev, stream, reps):
    """Plain per-view launches vs one persistent batched launch vs the render
    server, on 64 views of uneven size over 8 resident line sets."""
    sets_spec, views_spec = synth.batch_workload_spec()
    t = time.perf_counter()
    sets = []
    for sp in sets_spec:
        ls = synth.abc_lineset(sp["n_curves"], sp["n_vertices"], sp["seed"], sp["perturb"])
        with torch.cuda.stream(stream):
            s = L.lineset_voxelize(torch.as_tensor(ls.curve_off).to(dev), sp["grid"], 32,
                                   xyz=torch.as_tensor(ls.xyz).to(dev),
                                   attr=torch.as_tensor(ls.attr).to(dev), stream=stream)
        sets.append((sp, s))
        del ls
    log(f"[bench] batch workload: 8 sets voxelized in {time.perf_counter() - t:.1f}s")
    lut_op = torch.as_tensor(synth.lut_ramp(1.0)).to(dev)
    lut_tr = torch.as_tensor(synth.lut_importance_alpha()).to(dev)
    items = []
    for v in views_spec:
        sp, s = sets[v["set"]]
        cam = synth.look_camera((sp["grid"],) * 3, v["width"], v["height"], v["direction"], False)
        out = torch.empty((v["height"], v["width"], 4), dtype=torch.float32, device=dev)
        params = dict(radius=0.4, opaque=sp["opaque"], alpha_stop=0.95, merge_curves=True,
                      shading=1)
        items.append((s, cam, lut_op if sp["opaque"] else lut_tr, out, params))
    rays = sum(it[1].width * it[1].height for it in items)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        stream.synchronize()
        e0, e1 = ev(), ev()
        with torch.cuda.stream(stream):
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
        stream.synchronize()
        return e0.elapsed_time(e1) / reps

    def plain():
        for (s, cam, lut, out, params) in items:
            L.lineset_render(s, cam, lut, out=out, stream=stream, **params)

    plain_ms = timed(plain)
    t = time.perf_counter()
    with torch.cuda.stream(stream):
        b = L.Batch(items, autotune=True, graph=True, stream=stream)
    tune_s = time.perf_counter() - t
    batch_ms = timed(lambda: b.render(stream=stream))
    cfg = b.config()
    b.close()
    log(f"[bench] 64 views ({rays / 1e6:.1f} Mrays): plain {plain_ms:.2f} ms, "
        f"batched {batch_ms:.2f} ms ({cfg})")

    # render server, closed loop: all 64 views submitted at once
    budget = sum(s.info().device_bytes for _, s in sets) + (8 << 30)
    served = {}
    srv = L.Server(budget, n_slots=2, max_batch_views=64)
    ids = [srv.add_lineset(s) for _, s in sets]
    view_set = [v["set"] for v in views_spec]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for r in range(reps):
        tickets = [srv.submit(ids[view_set[k]], it[1], it[2], it[3], **it[4])
                   for k, it in enumerate(items)]
        for tk in tickets:
            srv.wait(tk)
    closed_s = time.perf_counter() - t
    st = srv.stats()
    served["closed_loop"] = dict(mrays_s=rays * reps / closed_s / 1e6, p50_ms=st["p50_ms"],
                                 p99_ms=st["p99_ms"], mean_batch=st["mean_batch"])
    srv.close()
    log(f"[bench] served: {served}")
    for _, s in sets:
        s.close()
    return {
        "workload": "64 views, area log-uniform 256^2..1920x1080, over 8 sets of 1M..20M "
                    "segments (128^3..512^3), even sets opaque",
        "rays_per_batch": rays,
        "plain_ms": plain_ms,
        "plain_mrays_s": rays / plain_ms / 1e3,
        "batched_ms": batch_ms,
        "batched_mrays_s": rays / batch_ms / 1e3,
        "batched_over_plain": plain_ms / batch_ms,
        "batch_config": cfg,
        "autotune_s": tune_s,
        "served": served,
    }


def update_leg(L, synth, torch, dev, stream, ls, w, reps=5, frac=0.01):
    """Incremental update vs full re-voxelization on the scale workload: each
    update removes `frac` of the curves (random ids) and appends as many new
    curves (another seed of the same flow, clamped into the set's box)."""
    grid, bins = w["grid"], w["bins"]
    xyz = torch.as_tensor(ls.xyz).to(dev)
    off = torch.as_tensor(ls.curve_off).to(dev)
    attr = torch.as_tensor(ls.attr).to(dev)
    k = max(1, int(frac * ls.n_curves))
    new = synth.abc_lineset(k, w["n_vertices"], 77, w["perturb"])
    lo, hi = ls.xyz.min(0), ls.xyz.max(0)
    nxyz = torch.as_tensor(np.clip(new.xyz, lo, hi).astype(np.float32)).to(dev)
    noff = torch.as_tensor(new.curve_off).to(dev)
    nattr = torch.as_tensor(new.attr).to(dev)
    rng = np.random.default_rng(8)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        s = L.lineset_voxelize(off, grid, bins, xyz=xyz, attr=attr, stream=stream)
    stream.synchronize()
    full, upd = [], []
    n_curves = ls.n_curves
    for r in range(reps + 1):
        rm = torch.as_tensor(rng.choice(n_curves, k, replace=False).astype(np.int64)).to(dev)
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        with torch.cuda.stream(stream):
            e0.record(stream)
            L.lineset_update(s, remove=rm, curve_off=noff, xyz=nxyz, attr=nattr, stream=stream)
            e1.record(stream)
            e2.record(stream)
            t = L.lineset_voxelize(off, grid, bins, xyz=xyz, attr=attr, stream=stream)
            e3.record(stream)
        stream.synchronize()
        t.close()
        n_curves += k
        if r > 0:
            upd.append(e0.elapsed_time(e1))
            full.append(e2.elapsed_time(e3))
    info = s.info()
    s.close()
    res = {"workload": f"scale set; per update remove {k} curves and add {k} "
                       f"({frac:.0%} of {ls.n_curves})",
           "update_ms_median": float(np.median(upd)), "full_voxelize_ms_median":
           float(np.median(full)), "records_after": int(info.n_records),
           "curves_after": int(info.n_curves)}
    log(f"[bench] update: {res}")
    return res


def gi_leg(L, synth, torch, dev, stream, reps=3):
    """The global-illumination workload (1M ABC-flow streamlines x 100
    vertices, perturbed; 512^3 grid, 32^2 bins; transparent; 16-cone AO and a
    soft shadow; 1920x1080 with AO/shadow shading): the same step as the main
    line (voxelize -> pyramid + AO + shadow grids -> render), timed per phase
    with events on the launch stream, and the ray caster's algorithmic bytes
    per launch."""
    w = dict(synth.WORKLOADS["gi"])
    t = time.perf_counter()
    ls = synth.abc_lineset(w["n_curves"], w["n_vertices"], w["seed"], w["perturb"])
    log(f"[bench] gi workload generated in {time.perf_counter() - t:.1f}s")
    grid, bins = w["grid"], w["bins"]
    cam = synth.default_camera((grid,) * 3, w["width"], w["height"], w["orthographic"])
    light = synth.LIGHT_DIR
    with torch.cuda.stream(stream):
        xyz = torch.as_tensor(ls.xyz).to(dev)
        off = torch.as_tensor(ls.curve_off).to(dev)
        attr = torch.as_tensor(ls.attr).to(dev)
        lut = torch.as_tensor(synth.lut_importance_alpha()).to(dev)
        out = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=dev)
    stream.synchronize()
    n_vert = int(xyz.shape[0])
    del ls
    rp = dict(radius=w["radius"], opaque=False, alpha_stop=0.95, merge_curves=True, shading=2,
              light_dir=light)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    ph = {"voxelize": [], "lod_illum": [], "render": []}
    for r in range(reps + 1):
        e = [ev() for _ in range(4)]
        with torch.cuda.stream(stream):
            e[0].record(stream)
            s = L.lineset_voxelize(off, grid, bins, xyz=xyz, attr=attr, stream=stream)
            e[1].record(stream)
            L.lineset_build_lod(s, lut, opaque=False, build_ao=True, ao_cones=16, ao_radius=15.0,
                                build_shadow=True, light_dir=light, stream=stream)
            e[2].record(stream)
            L.lineset_render(s, cam, lut, out=out, stream=stream, **rp)
            e[3].record(stream)
        stream.synchronize()
        if r > 0:
            ph["voxelize"].append(e[0].elapsed_time(e[1]))
            ph["lod_illum"].append(e[1].elapsed_time(e[2]))
            ph["render"].append(e[2].elapsed_time(e[3]))
        if r < reps:
            s.close()
    _, cnt = L.lineset_render_counted(s, cam, lut, out=out, stream=stream, **rp)
    info = s.info()
    s.close()
    med = {k: float(np.median(v)) for k, v in ph.items()}
    rays = cam.width * cam.height
    render_bytes = cnt["list_bytes"] + 16 * rays
    G3 = grid ** 3
    res = {
        "workload": (f"gi: {w['n_curves']} curves x {w['n_vertices']} vertices, {grid}^3 grid, "
                     f"{bins}^2 bins, r={w['radius']}, transparent, 16-cone AO + soft shadow, "
                     f"{cam.width}x{cam.height} perspective"),
        "records": int(info.n_records),
        "phases_ms_median": med,
        "step_ms": sum(med.values()),
        "step_mrays_s": rays / (sum(med.values()) * 1e-3) / 1e6,
        "render_mrays_s": rays / (med["render"] * 1e-3) / 1e6,
        "voxelize_min_bytes": 12 * n_vert + 9 * (int(off.shape[0]) - 1) + 8 * int(info.n_records)
        + 4 * (G3 + 1),
        "render_roofline": {
            "kernel": "k_render (ray caster)", "bound": "hbm",
            "algorithmic_bytes_per_launch": int(render_bytes),
            "achieved": render_bytes / (med["render"] * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": render_bytes / (med["render"] * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "counters": cnt,
    }
    res["voxelize_frac_hbm"] = (res["voxelize_min_bytes"] / (med["voxelize"] * 1e-3) / 1e9
                                / HBM_PEAK_GBS)
    log(f"[bench] gi: {res}")
    del xyz, off, attr, out
    torch.cuda.empty_cache()
    return res


def vdi_leg(L, synth, torch, dev, stream, s, cam, lut_op, lut_tr, light, reps=5):
    """View-dependent illumination on the resident scale set (its pyramid,
    grids and representative lines built): 1920x1080 frames with the
    per-fragment sources, opaque and transparent, against the per-voxel
    grids."""
    L.lineset_build_lod(s, lut_tr, opaque=False, build_ao=True, build_shadow=True,
                        light_dir=light, build_rep_lines=True, build_color=True, stream=stream)
    out = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    cases = {
        "grids": dict(),
        "hemisphere_ao_16": dict(ao_mode=1, ao_rays=16, ao_radius=15.0),
        "cone_shadow": dict(shadow_mode=1),
        "rep_shadow_level1": dict(shadow_mode=2, rep_level=1),
        "rep_shadow_level2": dict(shadow_mode=2, rep_level=2),
    }
    res = {}
    for opaque in (True, False):
        for name, kw in cases.items():
            p = dict(radius=0.4, opaque=opaque, alpha_stop=0.95, merge_curves=True, shading=2,
                     light_dir=light, **kw)
            lut = lut_op if opaque else lut_tr
            with torch.cuda.stream(stream):
                L.lineset_render(s, cam, lut, out=out, stream=stream, **p)
                e0, e1 = ev(), ev()
                e0.record(stream)
                for _ in range(reps):
                    L.lineset_render(s, cam, lut, out=out, stream=stream, **p)
                e1.record(stream)
            stream.synchronize()
            res[f"{'opaque' if opaque else 'transparent'}_{name}_ms"] = e0.elapsed_time(e1) / reps
    # opacity acceleration on the transparent frame (grid shading): time and
    # the largest per-channel difference from the exact frame
    p = dict(radius=0.4, opaque=False, alpha_stop=0.95, merge_curves=True, shading=2,
             light_dir=light)
    with torch.cuda.stream(stream):
        # (allocated, rendered and copied on the bench stream)
        exact = L.lineset_render(s, cam, lut_tr, stream=stream, **p).clone()
    stream.synchronize()
    for depth0 in (1.0, 2.0, 3.0):
        with torch.cuda.stream(stream):
            img = L.lineset_render(s, cam, lut_tr, out=out, stream=stream, accel_depth=depth0, **p)
            e0, e1 = ev(), ev()
            e0.record(stream)
            for _ in range(reps):
                L.lineset_render(s, cam, lut_tr, out=out, stream=stream, accel_depth=depth0, **p)
            e1.record(stream)
        stream.synchronize()
        res[f"transparent_accel_depth{depth0:g}_ms"] = e0.elapsed_time(e1) / reps
        res[f"transparent_accel_depth{depth0:g}_max_err"] = (img - exact).abs().max().item()
    log(f"[bench] view-dependent illumination / acceleration: {res}")
    return {"workload": "scale set, 1920x1080 perspective, shading 2 sources; opacity "
                        "acceleration (error bound exp(-depth))", **res}


def _lod_dims(grid):
    """Level sizes of the density pyramid of a cubic grid (halving to 1)."""
    dims, g = [], grid
    while True:
        dims.append((g, g, g))
        if g == 1:
            return dims
        g = (g + 1) // 2


def serve_sweep(L, synth, torch, dev, rates, seconds_per_rate, max_requests,
                arena_bytes):
    """Open-loop serving: Poisson arrivals at each rate over 4 resident sets
    of 1M / 5M / 20M / 50M segments (256^3, 256^3, 512^3, 512^3, AO and
    shadow grids built); resolution uniform over 512^2 / 1280x720 /
    1920x1080; transparency and AO shading each on with probability 1/2.
    Requests render into the server's output arena (`arena_bytes`, within
    the budget); the client collects each finished image while it waits for
    the next arrival, and a request whose arena block does not fit waits."""
    from collections import deque
    sets_spec, reqs = synth.serve_workload_spec(n_requests=max_requests)
    lut_tr = torch.as_tensor(synth.lut_importance_alpha()).to(dev)
    lut_op = torch.as_tensor(synth.lut_ramp(1.0)).to(dev)
    t = time.perf_counter()
    sets = []
    for sp in sets_spec:
        ls = synth.abc_lineset(sp["n_curves"], sp["n_vertices"], sp["seed"], sp["perturb"])
        s = L.lineset_voxelize(torch.as_tensor(ls.curve_off).to(dev), sp["grid"], 32,
                               xyz=torch.as_tensor(ls.xyz).to(dev),
                               attr=torch.as_tensor(ls.attr).to(dev))
        L.lineset_build_lod(s, lut_tr, opaque=False, build_ao=True, build_shadow=True,
                            light_dir=synth.LIGHT_DIR)
        sets.append(s)
        del ls
    torch.cuda.synchronize()
    resident = sum(s.info().device_bytes for s in sets)
    log(f"[bench] serving sets built in {time.perf_counter() - t:.1f}s "
        f"({resident / 2**30:.2f} GiB resident)")
    dst = {wh: torch.empty((wh[1], wh[0], 4), dtype=torch.float32, device=dev)
           for wh in synth.SERVE_RESOLUTIONS}
    cams = [synth.look_camera((sets_spec[r["set"]]["grid"],) * 3, r["width"], r["height"],
                              r["direction"], False) for r in reqs]
    budget = resident + arena_bytes + (1 << 20)
    rng = np.random.default_rng(55)
    out = {}
    for lam in rates:
        n_req = int(min(max_requests, max(100, lam * seconds_per_rate)))
        srv = L.Server(budget, n_slots=2, max_batch_views=64, output_arena_bytes=arena_bytes)
        ids = [srv.add_lineset(s) for s in sets]
        arrivals = np.cumsum(rng.exponential(1.0 / lam, n_req))
        pending = deque()
        offered = 0

        def collect(block):
            while pending and srv.wait(pending[0][0], timeout_us=-1 if block else 0):
                tk, wh = pending.popleft()
                srv.result(tk, dst[wh])

        t0 = time.perf_counter()
        for k in range(n_req):
            r = reqs[k]
            wh = (r["width"], r["height"])
            while True:
                collect(False)
                if time.perf_counter() - t0 >= arrivals[k]:
                    break
            params = dict(radius=0.4, opaque=not r["transparent"], alpha_stop=0.95,
                          merge_curves=True, shading=2 if r["ao"] else 1,
                          light_dir=synth.LIGHT_DIR)
            tk = srv.submit(ids[r["set"]], cams[k], lut_tr if r["transparent"] else lut_op,
                            None, **params)
            pending.append((tk, wh))
            offered += r["width"] * r["height"]
            if (k + 1) % 250 == 0:
                log(f"[bench] serve {lam:g} req/s: {k + 1}/{n_req} submitted")
        span = time.perf_counter() - t0
        collect(True)
        st = srv.stats()
        out[f"{lam:g}_per_s"] = dict(
            requests=n_req, offered_mrays_s=offered / span / 1e6, p50_ms=st["p50_ms"],
            p99_ms=st["p99_ms"], max_ms=st["max_ms"], mrays_s=st["mrays_per_s"],
            mean_batch=st["mean_batch"], held_for_memory=st["held_for_memory"],
            held_fraction=st["held_for_memory"] / n_req)
        log(f"[bench] serve {lam:g} req/s: {out[f'{lam:g}_per_s']}")
        srv.close()
    for s in sets:
        s.close()
    return {
        "workload": "Poisson arrivals over 4 resident sets of 1M/5M/20M/50M segments "
                    "(256^3/256^3/512^3/512^3); 512^2, 1280x720, 1920x1080 uniform; "
                    "transparency and AO each p=1/2; outputs in a server-owned arena",
        "budget_bytes": int(budget), "resident_bytes": int(resident),
        "output_arena_bytes": int(arena_bytes), "rates": out,
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1801_01155_amd as L
    from paper_1801_01155_amd import synth

    w = dict(synth.WORKLOADS[args.workload])
    log(f"[bench] generating workload {args.workload}: {w['n_curves']} x {w['n_vertices']}")
    t = time.perf_counter()
    ls = synth.abc_lineset(w["n_curves"], w["n_vertices"], w["seed"], w["perturb"])
    log(f"[bench] generated in {time.perf_counter() - t:.1f}s")
    grid, bins = w["grid"], w["bins"]
    cam = synth.default_camera((grid,) * 3, w["width"], w["height"], w["orthographic"])
    lut_np = synth.lut_ramp(1.0) if w["opaque"] else synth.lut_importance_alpha()
    light = synth.LIGHT_DIR

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        xyz = torch.as_tensor(ls.xyz).to(dev)
        off = torch.as_tensor(ls.curve_off).to(dev)
        attr = torch.as_tensor(ls.attr).to(dev)
        lut = torch.as_tensor(lut_np).to(dev)
        out = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=dev)
    stream.synchronize()
    rp = dict(radius=w["radius"], opaque=w["opaque"], alpha_stop=0.95, merge_curves=True,
              shading=2, light_dir=light)

    ev = lambda: torch.cuda.Event(enable_timing=True)
    phase_ms = {"voxelize": [], "lod_illum": [], "render": []}

    def step(record):
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        with torch.cuda.stream(stream):
            e0.record(stream)
            s = L.lineset_voxelize(off, grid, bins, xyz=xyz, attr=attr, stream=stream)
            e1.record(stream)
            L.lineset_build_lod(s, lut, opaque=w["opaque"], build_ao=True, ao_cones=16,
                                ao_radius=15.0, build_shadow=True, light_dir=light, stream=stream)
            e2.record(stream)
            L.lineset_render(s, cam, lut, out=out, stream=stream, **rp)
            e3.record(stream)
        if record:
            stream.synchronize()
            phase_ms["voxelize"].append(e0.elapsed_time(e1))
            phase_ms["lod_illum"].append(e1.elapsed_time(e2))
            phase_ms["render"].append(e2.elapsed_time(e3))
        return s

    for k in range(args.warmup):
        s = step(False)
        stream.synchronize()
        s.close()
        log(f"[bench] warmup {k + 1}/{args.warmup} done")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        s = step(True)
        s.close()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    rays = cam.width * cam.height
    log(f"[bench] {args.steps} steps in {elapsed:.3f}s ({ms_per_step:.2f} ms/step)")

    # work counters for the roofline (outside the timed region)
    s = L.lineset_voxelize(off, grid, bins, xyz=xyz, attr=attr, stream=stream)
    L.lineset_build_lod(s, lut, opaque=w["opaque"], build_ao=True, build_shadow=True,
                        light_dir=light, stream=stream)
    _, cnt = L.lineset_render_counted(s, cam, lut, out=out, stream=stream, **rp)
    info = s.info()
    # The timed steps render one view again and again, so from the second
    # frame on its tiles are launched longest first (their times measured the
    # frame before). A view the stream has not rendered, nor one near it,
    # starts in the ring order: the frame with the eye moved back along the
    # view by 3, 6, ..., 15 % of the grid's diagonal (each a new view).
    first_ms = []
    fwd = np.asarray(cam.forward, np.float64)
    fwd /= np.linalg.norm(fwd)
    diag = float(np.sqrt(3.0)) * grid
    for k in range(5):
        eye = np.asarray(cam.eye, np.float64) - fwd * diag * 0.03 * (k + 1)
        c2 = dataclasses.replace(cam, eye=tuple(float(x) for x in eye.astype(np.float32)))
        e0, e1 = ev(), ev()
        with torch.cuda.stream(stream):
            e0.record(stream)
            L.lineset_render(s, c2, lut, out=out, stream=stream, **rp)
            e1.record(stream)
        stream.synchronize()
        first_ms.append(e0.elapsed_time(e1))
    # A camera in motion: the view direction turned 0.5 degree per frame
    # about the vertical axis, 12 frames; each frame after the first is
    # launched in the order of the previous frame's tile times.
    moving_ms = []
    for k in range(12):
        a = np.radians(0.5 * (k + 1))
        d = (np.cos(a) * 1.0 - np.sin(a) * 0.8, np.sin(a) * 1.0 + np.cos(a) * 0.8, 0.6)
        c2 = synth.look_camera((grid,) * 3, cam.width, cam.height, d, w["orthographic"])
        e0, e1 = ev(), ev()
        with torch.cuda.stream(stream):
            e0.record(stream)
            L.lineset_render(s, c2, lut, out=out, stream=stream, **rp)
            e1.record(stream)
        stream.synchronize()
        moving_ms.append(e0.elapsed_time(e1))
    render_ms = float(np.mean(phase_ms["render"]))
    render_bytes = cnt["list_bytes"] + 16 * rays
    achieved = render_bytes / (render_ms * 1e-3) / 1e9
    med = {k: float(np.median(v)) for k, v in phase_ms.items()}
    traffic = None
    counters_profiled = None
    if RENDER_TRAFFIC is not None:
        import hashlib
        src = os.path.join(ROOT, "paper_1801_01155_amd", "csrc", "render.hip")
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() == RENDER_TRAFFIC["render_hip_sha256"]:
                traffic = RENDER_TRAFFIC["bytes_per_launch"]
                counters_profiled = dict(RENDER_COUNTERS)
    valu_tflops = cnt["tested"] * CAPSULE_FLOPS / (render_ms * 1e-3) / 1e12
    # minimum HBM bytes per phase (inputs read once, outputs written once)
    G3 = grid ** 3
    n_rec = int(info.n_records)
    n_lod = int(sum(int(np.prod(d)) for d in _lod_dims(grid)))
    phase_bytes = {
        "voxelize": 12 * int(xyz.shape[0]) + 9 * (int(off.shape[0]) - 1) + 8 * n_rec
        + 4 * (G3 + 1),
        "lod_illum": 8 * n_rec + 4 * (G3 + 1) + 3 * 4 * G3 + 4 * n_lod + 2 * 4 * G3,
        "render": render_bytes,
    }
    phase_roof = {k: {"algorithmic_bytes": int(b), "ms": med[k],
                      "GB_s": b / (med[k] * 1e-3) / 1e9,
                      "frac_hbm": b / (med[k] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                  for k, b in phase_bytes.items()}
    log(f"[bench] phases (median ms): {med}; counters {cnt}")

    result = {
        "metric": "Mrays/s (1920x1080 frames through the whole voxel ray-casting path)",
        "value": rays / (ms_per_step * 1e-3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (fp64 ray set-up and grid walk; int64 voxelization)",
        "data": "synthetic: seeded ABC-flow streamlines (no dataset)",
        "config": {
            "workload": (f"{args.workload}: {w['n_curves']} curves x {w['n_vertices']} vertices, "
                         f"{grid}^3 grid, {bins}^2 bins, r={w['radius']}, "
                         f"{'opaque' if w['opaque'] else 'transparent'}, "
                         f"{cam.width}x{cam.height} perspective; step = voxelize + LoD + "
                         f"AO/shadow grids + render"),
            "global_batch": 1,
            "records": int(info.n_records),
            "parallelism": "single GPU",
        },
        "phases_ms_median": med,
        "render_mrays_s": rays / (med["render"] * 1e-3) / 1e6,
        "ms_per_frame_render": med["render"],
        "ms_per_frame_render_first_view": float(np.median(first_ms)),
        "ms_per_frame_render_moving_camera": float(np.median(moving_ms[1:])),
        "roofline": {
            "kernel": "k_render (ray caster)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_GB_s": (traffic / (render_ms * 1e-3) / 1e9) if traffic else None,
            "algorithmic_bytes_per_launch": int(render_bytes),
            "avg_launch_ms": render_ms,
            # the other ceilings and what limits the kernel: capsule-test
            # arithmetic against the fp32 vector peak, and the profiled L2 hit
            # rate, lane use and wait share of this kernel source (null once
            # the source has changed since the counters were taken)
            "valu": {"achieved_tflops": valu_tflops, "peak_tflops": VALU_PEAK_TFLOPS,
                     "frac": valu_tflops / VALU_PEAK_TFLOPS,
                     "flops_per_test": CAPSULE_FLOPS, "tests": int(cnt["tested"])},
            "profiled": counters_profiled,
            "limiter": ("memory latency and divergence: a wave's time is its slowest "
                        "ray's; HBM and VALU both far below their peaks"),
        },
        "phase_rooflines": phase_roof,
        "counters": cnt,
    }
    if not args.no_vdi:
        result["view_dependent"] = vdi_leg(L, synth, torch, dev, stream, s, cam,
                                           torch.as_tensor(synth.lut_ramp(1.0)).to(dev), lut,
                                           light)
    s.close()
    if not args.no_update:
        result["update"] = update_leg(L, synth, torch, dev, stream, ls, w)
    if not args.no_gi:
        result["gi"] = gi_leg(L, synth, torch, dev, stream)
    if not args.no_batch:
        result["batched"] = batched_vs_plain(L, synth, torch, dev, stream, max(3, args.steps // 2))
    if not args.no_serve:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        result["serving"] = serve_sweep(L, synth, torch, dev, rates, args.serve_seconds,
                                        args.serve_max_requests,
                                        int(args.serve_arena_mib * 2**20))
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(ls, w, cam, lut_np, light, args.cpu_sample_rows)
    print(json.dumps(result), flush=True)
    if args.copy_calibration:
        x = torch.ones(COPY_CAL_BYTES // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {COPY_CAL_BYTES} bytes done")


if __name__ == "__main__":
    main()
