"""Writes tests/golden/oracle_small.json: the oracle's results on the small
streamline workload (1000 ABC-flow curves x 64 vertices, 64^3 grid, 32^2 bins,
opaque, 256x256 orthographic). Calls only the oracle (and the seeded input
generator). The file is a regression pin of the oracle: a change to its
arithmetic that moves these values must name the passage of the paper that
justifies it.

    python tests/golden/make_oracle_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1801_01155_amd import synth  # noqa: E402

SAMPLE_PIXELS = [0, 777, 12345, 20000, 30000, 32896, 40000, 45678, 50000, 65535]


def compute():
    w = synth.WORKLOADS["small"]
    ls = synth.abc_lineset(w["n_curves"], w["n_vertices"], w["seed"])
    lat, _, _ = O.grid_setup(ls.xyz, w["grid"])
    csr = O.voxelize(lat, ls.curve_off, ls.attr, w["grid"], w["bins"])
    cam = synth.default_camera((w["grid"],) * 3, w["width"], w["height"], orthographic=True)
    img, cnt = O.render(csr, w["grid"], w["bins"], cam, lut=synth.lut_ramp(1.0),
                        radius=w["radius"], opaque=True, shading=1)
    _, _, rho, _, _ = O.lod(csr, w["grid"], w["bins"], synth.lut_ramp(1.0), opaque=True)
    flat = img.reshape(-1, 4)
    return {
        "workload": "small: 1000 x 64 ABC-flow curves (seed 1), 64^3, N=32, r=0.4, opaque, "
                    "256x256 orthographic, headlight shading",
        "n_records": int(len(csr.records)),
        "offsets_sha256": hashlib.sha256(csr.offsets.astype("<u4").tobytes()).hexdigest(),
        "records_sha256": hashlib.sha256(csr.records.astype("<u8").tobytes()).hexdigest(),
        "rho_sum": float(rho.sum()),
        "image_channel_sums": [float(x) for x in flat.sum(0)],
        "covered_pixels": int((flat[:, 3] > 0).sum()),
        "sample_pixels": SAMPLE_PIXELS,
        "sample_values": [[float(x) for x in flat[k]] for k in SAMPLE_PIXELS],
        "counters": {k: int(v) for k, v in cnt.items()},
    }


if __name__ == "__main__":
    out = os.path.join(HERE, "oracle_small.json")
    with open(out, "w") as f:
        json.dump(compute(), f, indent=1)
    print("wrote", out)
