"""Brute-force voxelizer in exact rational arithmetic (fractions.Fraction).

An independent second derivation of the per-voxel line lists (sections
"Curve voxelization" and "Line quantization"), used only to pin the oracle on
tiny inputs. It shares no code with the oracle and works differently: plane
crossings are enumerated per axis and grouped by their exact parameter in a
dict, and the voxel entered at each event is found by flooring the exact
curve point half-way to the next event (or the segment's end vertex), not by
stepping cell indices.
"""
from fractions import Fraction
from math import floor


def _cell_at(P0, P1, t):
    return tuple(floor((P0[a] + t * (P1[a] - P0[a])) / 256) for a in range(3))


def _face_bins(axis, point, cell, bins):
    others = [b for b in range(3) if b != axis]
    out = []
    for b in others:
        local = (point[b] - 256 * cell[b]) / Fraction(256)
        assert 0 <= local <= 1
        out.append(min(floor(local * bins), bins - 1))
    return out


def _code(face, bu, bw):
    return face | (bu << 3) | (bw << 9)


def curve_records(verts, bins, vattr=None):
    """verts: list of integer (x, y, z) lattice points. Returns a list of
    (voxel_cell, entry_code, exit_code) in order along the curve; with
    per-vertex attributes vattr, (voxel_cell, entry_code, exit_code,
    entry_attr, exit_attr), an event's attribute being a_i + (a_{i+1} - a_i) t
    rounded half up (t the exact parameter of the event on its segment)."""
    if len(verts) < 2:
        return []
    events = []  # (point (Fractions), exit_code_old_cell, entry_code_new_cell, old, new)
    cell = tuple(v // 256 for v in verts[0])
    for i in range(len(verts) - 1):
        P0, P1 = verts[i], verts[i + 1]
        crossings = {}
        for a in range(3):
            lo, hi = sorted((P0[a], P1[a]))
            for k in range(lo // 256 - 1, hi // 256 + 2):
                plane = 256 * k
                up = P0[a] < plane <= P1[a]
                down = P1[a] < plane <= P0[a]
                if up or down:
                    t = Fraction(plane - P0[a], P1[a] - P0[a])
                    crossings.setdefault(t, []).append(a)
        ts = sorted(crossings)
        for n, t in enumerate(ts):
            if t == 1:
                new = tuple(v // 256 for v in P1)
            else:
                t_next = ts[n + 1] if n + 1 < len(ts) else Fraction(1)
                new = _cell_at(P0, P1, (t + t_next) / 2)
            changed = [a for a in range(3) if new[a] != cell[a]]
            assert sorted(changed) == sorted(crossings[t])
            fa = min(changed)
            up = new[fa] > cell[fa]
            point = tuple(P0[b] + t * (P1[b] - P0[b]) for b in range(3))
            exit_face = 2 * fa + (1 if up else 0)
            entry_face = 2 * fa + (0 if up else 1)
            ex = _code(exit_face, *_face_bins(fa, point, cell, bins))
            en = _code(entry_face, *_face_bins(fa, point, new, bins))
            at = None
            if vattr is not None:
                at = floor(vattr[i] + t * (vattr[i + 1] - vattr[i]) + Fraction(1, 2))
            events.append((point, ex, en, cell, new, at))
            cell = new
    assert cell == tuple(v // 256 for v in verts[-1])
    recs = []
    for j in range(len(events) - 1):
        p0, _, entry, _, c_in, a_in = events[j]
        p1, exit_, _, c_out, _, a_out = events[j + 1]
        assert c_in == c_out
        if p0 == p1 or entry == exit_:
            continue
        recs.append((c_in, entry, exit_) if vattr is None else (c_in, entry, exit_, a_in, a_out))
    return recs


def voxelize(lattice, curve_off, attr, grid, bins, vattr=None):
    """Returns (offsets list, records list) in the oracle's CSR format; with
    per-vertex attributes also the per-record endpoint attributes
    (entry | exit << 8) and the records' attribute byte their mean."""
    gx, gy, gz = grid
    items = []
    for c in range(len(curve_off) - 1):
        verts = [tuple(int(x) for x in lattice[v]) for v in range(curve_off[c], curve_off[c + 1])]
        va = None if vattr is None else [int(vattr[v]) for v in range(curve_off[c], curve_off[c + 1])]
        a = 255 if attr is None else int(attr[c])
        for r in curve_records(verts, bins, va):
            (cx, cy, cz), entry, exit_ = r[:3]
            ends = 0
            aa = a
            if va is not None:
                aa = (r[3] + r[4]) // 2
                ends = r[3] | (r[4] << 8)
            vox = cx + gx * (cy + gy * cz)
            rec = entry | (exit_ << 15) | (aa << 32) | ((c & 0xFFFFFF) << 40)
            items.append((vox, len(items), rec, ends))
    items.sort()
    nvox = gx * gy * gz
    counts = [0] * (nvox + 1)
    for it in items:
        counts[it[0] + 1] += 1
    for v in range(nvox):
        counts[v + 1] += counts[v]
    if vattr is None:
        return counts, [it[2] for it in items]
    return counts, [it[2] for it in items], [it[3] for it in items]
