"""Representative lines by brute force in exact rational arithmetic.

An independent second derivation of the per-voxel representative lines of
section "LoD construction", used only to pin the oracle on tiny inputs. It
shares no code with the oracle and works differently: endpoints are
fractions.Fraction points in voxel units, and each average point is snapped
by scanning every bin centre of all six faces (the oracle reduces the scan to
one closest bin per axis and face in scaled integers).

Reading (the same one the oracle documents): per voxel, lines in list order,
each flipped when its direction has a negative dot product with the previous
(possibly flipped) line; start and end points averaged separately; each
average snapped to the closest bin centre on the boundary (first face, then
lowest bins, on ties); two face-adjacent voxels both ending on their common
face (one endpoint each) move those endpoints to the bin of their mean (a
point on a bin boundary belongs to the upper bin); coarser levels repeat this
over the joined lines of the children (x fastest, then y, then z), in the
parent's frame.
"""
from fractions import Fraction
from math import floor

NONE = 0xFFFFFFFF


def _axes(face):
    axis = face >> 1
    others = [b for b in range(3) if b != axis]
    return axis, others[0], others[1]


def point_of(code15, bins):
    face = code15 & 7
    axis, ua, wa = _axes(face)
    p = [Fraction(0)] * 3
    p[axis] = Fraction(face & 1)
    p[ua] = (Fraction((code15 >> 3) & 63) + Fraction(1, 2)) / bins
    p[wa] = (Fraction((code15 >> 9) & 63) + Fraction(1, 2)) / bins
    return p


def snap(point, bins):
    best, code = None, None
    for face in range(6):
        axis, ua, wa = _axes(face)
        for bu in range(bins):
            for bw in range(bins):
                c = [Fraction(0)] * 3
                c[axis] = Fraction(face & 1)
                c[ua] = (Fraction(bu) + Fraction(1, 2)) / bins
                c[wa] = (Fraction(bw) + Fraction(1, 2)) / bins
                d2 = sum((point[k] - c[k]) ** 2 for k in range(3))
                if best is None or d2 < best:
                    best, code = d2, face | (bu << 3) | (bw << 9)
    return code


def average_line(lines, bins):
    """lines: list of (start, end) Fraction points in the voxel's frame."""
    if not lines:
        return NONE
    S, E = [Fraction(0)] * 3, [Fraction(0)] * 3
    prev = None
    for a, b in lines:
        d = [b[k] - a[k] for k in range(3)]
        if prev is not None and sum(d[k] * prev[k] for k in range(3)) < 0:
            a, b = b, a
            d = [-x for x in d]
        S = [S[k] + a[k] for k in range(3)]
        E = [E[k] + b[k] for k in range(3)]
        prev = d
    n = len(lines)
    s = snap([x / n for x in S], bins)
    e = snap([x / n for x in E], bins)
    return s | (e << 15)


def connect(pre, dims, bins):
    """pre: dict cell -> code (absent = none). Returns the joined dict."""
    out = {}
    for cell, code in pre.items():
        ends = [code & 0x7FFF, (code >> 15) & 0x7FFF]
        if (ends[0] & 7) != (ends[1] & 7):
            for e in range(2):
                face = ends[e] & 7
                axis = face >> 1
                nb = list(cell)
                nb[axis] += 1 if face & 1 else -1
                nb = tuple(nb)
                if nb not in pre:
                    continue
                m = pre[nb]
                n_ends = [m & 0x7FFF, (m >> 15) & 0x7FFF]
                on = [x for x in n_ends if (x & 7) == (face ^ 1)]
                if len(on) != 1:
                    continue
                mine, other = point_of(ends[e], bins), point_of(on[0], bins)
                _, ua, wa = _axes(face)
                mid_u = (mine[ua] + other[ua]) / 2
                mid_w = (mine[wa] + other[wa]) / 2
                bu = min(floor(mid_u * bins), bins - 1)
                bw = min(floor(mid_w * bins), bins - 1)
                ends[e] = face | (bu << 3) | (bw << 9)
        out[cell] = ends[0] | (ends[1] << 15)
    return out


def rep_levels(offsets, records, grid, bins):
    """Returns a list of dicts (cell -> code), one per level, finest first."""
    gx, gy, gz = grid
    pre = {}
    for z in range(gz):
        for y in range(gy):
            for x in range(gx):
                v = x + gx * (y + gy * z)
                lines = [(point_of(int(r) & 0x7FFF, bins), point_of((int(r) >> 15) & 0x7FFF, bins))
                         for r in records[offsets[v]:offsets[v + 1]]]
                if lines:
                    pre[(x, y, z)] = average_line(lines, bins)
    dims = [tuple(grid)]
    levels = [connect(pre, dims[0], bins)]
    while dims[-1] != (1, 1, 1):
        child, cd = levels[-1], dims[-1]
        pd = tuple((d + 1) // 2 for d in cd)
        pre = {}
        for z in range(pd[2]):
            for y in range(pd[1]):
                for x in range(pd[0]):
                    lines = []
                    for k in range(8):
                        off = (k & 1, (k >> 1) & 1, k >> 2)
                        c = (2 * x + off[0], 2 * y + off[1], 2 * z + off[2])
                        if c not in child:
                            continue
                        code = child[c]
                        a = point_of(code & 0x7FFF, bins)
                        b = point_of((code >> 15) & 0x7FFF, bins)
                        lines.append(([(off[q] + a[q]) / 2 for q in range(3)],
                                      [(off[q] + b[q]) / 2 for q in range(3)]))
                    if lines:
                        pre[(x, y, z)] = average_line(lines, bins)
        dims.append(pd)
        levels.append(connect(pre, pd, bins))
    return levels, dims
