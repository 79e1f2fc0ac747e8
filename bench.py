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
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


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
    return ap.parse_args()


def cpu_baseline(ls, w, cam, lut, light, row_stride):
    """The oracle, untuned, on the host cores: voxelize a 10% curve sample,
    LoD + AO + shadow grids in full, render every row_stride-th row; scaled
    to one full step."""
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    grid, bins = w["grid"], w["bins"]
    sub = max(1, ls.n_curves // 10)
    off = ls.curve_off[:sub + 1]
    t = time.perf_counter()
    lat, _, _ = O.grid_setup(ls.xyz[:off[-1]], grid)
    O.voxelize(lat, off, ls.attr[:sub], grid, bins)
    t_vox = (time.perf_counter() - t) * (ls.n_curves / sub)
    # full CSR for the later stages (not timed)
    lat, _, _ = O.grid_setup(ls.xyz, grid)
    csr = O.voxelize(lat, ls.curve_off, ls.attr, grid, bins)
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
    return {
        "value": W * H / step / 1e6,
        "unit": "Mrays/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"voxelize {sub} of {ls.n_curves} curves (x{ls.n_curves / sub:.0f}); "
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

    # render server: closed loop (all 64 views submitted at once), then an
    # open-loop Poisson probe
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
    rng = np.random.default_rng(5)
    for lam in (100.0, 400.0):
        srv = L.Server(budget, n_slots=2, max_batch_views=64)
        ids = [srv.add_lineset(s) for _, s in sets]
        n_req = int(lam * 1.0)
        outs = [torch.empty_like(items[k % len(items)][3]) for k in range(n_req)]
        arrivals = np.cumsum(rng.exponential(1.0 / lam, n_req))
        t0 = time.perf_counter()
        tickets = []
        for k in range(n_req):
            while time.perf_counter() - t0 < arrivals[k]:
                pass
            it = items[k % len(items)]
            tickets.append(srv.submit(ids[view_set[k % len(items)]], it[1], it[2], outs[k], **it[4]))
        for tk in tickets:
            srv.wait(tk)
        st = srv.stats()
        served[f"poisson_{int(lam)}_per_s"] = dict(requests=n_req, p50_ms=st["p50_ms"],
                                                  p99_ms=st["p99_ms"], mean_batch=st["mean_batch"],
                                                  mrays_s=st["mrays_per_s"])
        srv.close()
        del outs
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


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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
    render_ms = float(np.mean(phase_ms["render"]))
    render_bytes = cnt["list_bytes"] + 16 * rays
    achieved = render_bytes / (render_ms * 1e-3) / 1e9
    med = {k: float(np.median(v)) for k, v in phase_ms.items()}
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
        "roofline": {
            "kernel": "k_render (ray caster)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes_per_launch": int(render_bytes),
            "avg_launch_ms": render_ms,
        },
        "counters": cnt,
    }
    s.close()
    if not args.no_batch:
        result["batched"] = batched_vs_plain(L, synth, torch, dev, stream, max(3, args.steps // 2))
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(ls, w, cam, lut_np, light, args.cpu_sample_rows)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
