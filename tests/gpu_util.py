"""Shared helpers for the GPU parity tests: run the HIP path and the oracle
on the same seeded inputs and compare."""
import numpy as np
import torch

import oracle as O
import paper_1801_01155_amd as L
from paper_1801_01155_amd import synth

IMAGE_TOL = 2e-3          # max per-channel abs error ...
IMAGE_FRACTION = 0.999    # ... on at least this fraction of pixels


def gpu_csr(ls):
    offs = L.lineset_export(ls, L.EXPORT_OFFSETS).cpu().numpy().view(np.uint32)
    recs = L.lineset_export(ls, L.EXPORT_RECORDS).cpu().numpy().view(np.uint64)
    return offs, recs


def image_report(gpu_img, ref_img, label=""):
    """Max abs error and fraction of pixels within IMAGE_TOL (all channels)."""
    g = np.asarray(gpu_img, dtype=np.float64).reshape(-1, 4)
    r = np.asarray(ref_img, dtype=np.float64).reshape(-1, 4)
    err = np.abs(g - r).max(axis=1)
    frac = float((err <= IMAGE_TOL).mean())
    print(f"[image {label}] pixels={len(err)} max_abs_err={err.max():.3e} "
          f"frac_within_{IMAGE_TOL:g}={frac:.6f} worst_px={int(err.argmax())}", flush=True)
    return float(err.max()), frac


def assert_image_parity(gpu_img, ref_img, label=""):
    mx, frac = image_report(gpu_img, ref_img, label)
    assert frac >= IMAGE_FRACTION, f"{label}: only {frac:.5f} of pixels within {IMAGE_TOL}"
    return mx, frac


def workload(name, **over):
    w = dict(synth.WORKLOADS[name])
    w.update(over)
    ls = synth.abc_lineset(w["n_curves"], w["n_vertices"], w["seed"], w["perturb"])
    return w, ls


def oracle_csr_from_xyz(ls, grid, bins):
    lat, lo, s = O.grid_setup(ls.xyz, grid)
    return O.voxelize(lat, ls.curve_off, ls.attr, grid, bins), lat


def lut_for(w):
    return synth.lut_ramp(1.0) if w["opaque"] else synth.lut_importance_alpha()


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()
