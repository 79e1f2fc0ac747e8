"""Brute-force ray casters for tiny inputs.

render: every ray against every capsule, one global sort. Pins the oracle's
neighbour-voxel mode (section "Ray-tube intersections": with the lines of
adjacent voxels included, every tube piece a ray meets is found). No grid
traversal at all.

render_own_voxel: the own-voxel mode written from its definition without a
grid walk: the voxels the ray meets are found by testing every voxel's box
(sorted by entry parameter); in that order each voxel's own lines that the
ray hits in front of its origin (t_in >= 0, anywhere along the ray) are
composited, nearest entry first.

In both the capsule interval is found numerically from the convex distance
function f(t) = dist(o + t d, segment) - r (minimum by golden-section
search, the two roots by bisection), independently of the oracle's closed
forms.
"""
import numpy as np


def decode(rec, bins):
    """Record -> (entry, exit) local points; an independent decoder."""
    def one(code):
        face = code & 7
        axis, side = face >> 1, face & 1
        inplane = [b for b in range(3) if b != axis]
        p = np.zeros(3)
        p[axis] = side
        p[inplane[0]] = (((code >> 3) & 63) + 0.5) / bins
        p[inplane[1]] = (((code >> 9) & 63) + 0.5) / bins
        return p
    rec = int(rec)
    return one(rec & 0x7FFF), one((rec >> 15) & 0x7FFF)


def ray_for_pixel(cam, i, j):
    e, f, r, u = [np.asarray(x, dtype=np.float64) for x in cam.as_arrays()]
    uu = (2.0 * (i + 0.5)) / cam.width - 1.0
    vv = 1.0 - (2.0 * (j + 0.5)) / cam.height
    if cam.orthographic:
        o = (e + uu * r) + vv * u
        d = f
    else:
        o = e
        d = (f + uu * r) + vv * u
    return o.astype(np.float32).astype(np.float64), d.astype(np.float32).astype(np.float64)


def _seg_dist(P, A, B):
    ba = B - A
    u = np.clip(((P - A) * ba).sum(-1) / (ba * ba).sum(-1), 0.0, 1.0)
    return np.linalg.norm(P - (A + u[..., None] * ba), axis=-1)


def capsule_intervals(o, d, A, B, r, t_lo, t_hi, iters=200):
    """Vectorised over capsules: (hit mask, t_in, t_out) on [t_lo, t_hi]."""
    f = lambda t: _seg_dist(o + t[:, None] * d, A, B) - r
    a = np.full(len(A), float(t_lo))
    b = np.full(len(A), float(t_hi))
    g = (np.sqrt(5.0) - 1.0) / 2.0
    for _ in range(iters):
        c = b - g * (b - a)
        e = a + g * (b - a)
        left = f(c) < f(e)
        b = np.where(left, e, b)
        a = np.where(left, a, c)
    tm = 0.5 * (a + b)
    hit = f(tm) <= 0
    lo = np.full(len(A), float(t_lo))
    hi = tm.copy()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        inside = f(mid) <= 0
        hi = np.where(inside, mid, hi)
        lo = np.where(inside, lo, mid)
    t_in = hi
    lo = tm.copy()
    hi = np.full(len(A), float(t_hi))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        inside = f(mid) <= 0
        lo = np.where(inside, mid, lo)
        hi = np.where(inside, hi, mid)
    t_out = lo
    return hit, t_in, t_out


def clip_box(o, d, grid):
    t0, t1 = 0.0, np.inf
    for a in range(3):
        if d[a] != 0:
            ta, tb = (0 - o[a]) / d[a], (grid[a] - o[a]) / d[a]
            t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
        elif not (0 <= o[a] < grid[a]):
            return None
    return (t0, t1) if t0 < t1 else None


def render(offsets, records, grid, bins, cam, lut, radius, opaque, alpha_stop,
           merge_curves, shading, ka=0.25, kd=0.75, ks=0.2, shininess=16.0, pixels=None):
    gx, gy, gz = grid
    n = len(records)
    A = np.zeros((n, 3))
    B = np.zeros((n, 3))
    owner = np.repeat(np.arange(len(offsets) - 1), np.diff(np.asarray(offsets, dtype=np.int64)))
    for k in range(n):
        v = int(owner[k])
        cell = np.array([v % gx, (v // gx) % gy, v // (gx * gy)], dtype=np.float64)
        ea, eb = decode(records[k], bins)
        A[k] = cell + ea
        B[k] = cell + eb
    W, H = cam.width, cam.height
    pix = range(W * H) if pixels is None else pixels
    out = np.zeros((len(pix), 4))
    for m, p in enumerate(pix):
        i, j = p % W, p // W
        o, d = ray_for_pixel(cam, i, j)
        box = clip_box(o, d, grid)
        if box is None or n == 0:
            continue
        span = box[1] - box[0]
        hit, tin, tout = capsule_intervals(o, d, A, B, radius, box[0] - span, box[1] + span)
        keep = np.nonzero(hit & (tin >= box[0]) & (tin < box[1]))[0]
        order = sorted(keep, key=lambda k: (tin[k], k))
        out[m] = _composite(order, records, A, B, tin, tout, o, d, lut, opaque, alpha_stop,
                            merge_curves, shading, ka, kd, ks, shininess)
    return out


def _composite(order, records, A, B, tin, tout, o, d, lut, opaque, alpha_stop, merge_curves,
               shading, ka, kd, ks, shininess):
    """Front-to-back compositing of the hits in `order` (record indices);
    a curve's hit starting inside its open interval only extends it."""
    C = np.zeros(3)
    acc = 0.0
    opened = {}
    vdir = -d / np.linalg.norm(d)
    for k in order:
        rec = int(records[k])
        tag, attr = rec >> 40, (rec >> 32) & 0xFF
        if not opaque and merge_curves:
            if tag in opened and tin[k] <= opened[tag]:
                opened[tag] = max(opened[tag], tout[k])
                continue
            opened[tag] = tout[k]
        rgb = np.asarray(lut[attr][:3], dtype=np.float64)
        alpha = 1.0 if opaque else float(lut[attr][3])
        if shading == 0:
            col = rgb
        else:
            P = o + tin[k] * d
            ba = B[k] - A[k]
            u = np.clip((P - A[k]) @ ba / (ba @ ba), 0, 1)
            nrm = P - (A[k] + u * ba)
            nrm = nrm / np.linalg.norm(nrm)
            ndv = abs(nrm @ vdir)
            col = rgb * (ka + kd * ndv) + ks * ndv ** shininess
        w = (1.0 - acc) * alpha
        C += w * col
        acc += w
        if acc >= alpha_stop:
            break
    return np.array([C[0], C[1], C[2], acc])


def _segments(offsets, records, grid, bins):
    gx, gy, gz = grid
    n = len(records)
    A = np.zeros((n, 3))
    B = np.zeros((n, 3))
    owner = np.repeat(np.arange(len(offsets) - 1), np.diff(np.asarray(offsets, dtype=np.int64)))
    for k in range(n):
        v = int(owner[k])
        cell = np.array([v % gx, (v // gx) % gy, v // (gx * gy)], dtype=np.float64)
        ea, eb = decode(records[k], bins)
        A[k] = cell + ea
        B[k] = cell + eb
    return A, B, owner


def voxels_met(o, d, grid):
    """Every voxel whose box the ray (t >= 0) crosses over a positive
    length, as (entry t, voxel id), sorted by entry."""
    gx, gy, gz = grid
    out = []
    for z in range(gz):
        for y in range(gy):
            for x in range(gx):
                lo, hi, ok = 0.0, np.inf, True
                for a, c in enumerate((x, y, z)):
                    if d[a] != 0:
                        ta, tb = (c - o[a]) / d[a], (c + 1 - o[a]) / d[a]
                        lo, hi = max(lo, min(ta, tb)), min(hi, max(ta, tb))
                    elif not (c <= o[a] < c + 1):
                        ok = False
                if ok and lo < hi:
                    out.append((lo, x + gx * (y + gy * z)))
    out.sort()
    return out


def render_own_voxel(offsets, records, grid, bins, cam, lut, radius, opaque, alpha_stop,
                     merge_curves, shading, ka=0.25, kd=0.75, ks=0.2, shininess=16.0):
    A, B, owner = _segments(offsets, records, grid, bins)
    n = len(records)
    W, H = cam.width, cam.height
    out = np.zeros((W * H, 4))
    for p in range(W * H):
        o, d = ray_for_pixel(cam, p % W, p // W)
        box = clip_box(o, d, grid)
        if box is None or n == 0:
            continue
        span = box[1] - box[0]
        hit, tin, tout = capsule_intervals(o, d, A, B, radius, box[0] - span, box[1] + span)
        order = []
        for _, v in voxels_met(o, d, grid):
            own = [k for k in range(int(offsets[v]), int(offsets[v + 1])) if hit[k] and tin[k] >= 0]
            order += sorted(own, key=lambda k: (tin[k], k))
        out[p] = _composite(order, records, A, B, tin, tout, o, d, lut, opaque, alpha_stop,
                            merge_curves, shading, ka, kd, ks, shininess)
    return out
