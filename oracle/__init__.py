"""Python access to the CPU oracle (``lineset_oracle.c``).

TEST INFRASTRUCTURE ONLY. Imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the product package. It shares
no code with the HIP library: this module only marshals numpy arrays into
the C oracle.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lineset_oracle.c")
_LIB = os.path.join(_HERE, "liblineset_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liblineset_oracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class Csr(C.Structure):
    _fields_ = [("n_records", C.c_int64), ("n_voxels", C.c_int64),
                ("offsets", C.POINTER(C.c_uint32)), ("records", C.POINTER(C.c_uint64)),
                ("n_events", C.c_int64), ("n_dropped", C.c_int64),
                ("ends", C.POINTER(C.c_uint16))]


class CameraS(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("forward", C.c_float * 3),
                ("right", C.c_float * 3), ("up", C.c_float * 3),
                ("orthographic", C.c_int32), ("width", C.c_int32), ("height", C.c_int32)]


class ParamsS(C.Structure):
    _fields_ = [("radius", C.c_float), ("mode", C.c_int32), ("opaque", C.c_int32),
                ("alpha_stop", C.c_float), ("merge_curves", C.c_int32),
                ("lut_rgba", C.POINTER(C.c_float)), ("shading", C.c_int32),
                ("ka", C.c_float), ("kd", C.c_float), ("ks", C.c_float),
                ("shininess", C.c_float), ("light_dir", C.c_float * 3),
                ("distance_alpha", C.c_int32), ("ao_mode", C.c_int32),
                ("shadow_mode", C.c_int32), ("ao_rays", C.c_int32), ("ao_radius", C.c_float),
                ("rep_level", C.c_int32), ("rho", C.POINTER(C.c_double)),
                ("rep", C.POINTER(C.c_uint32)), ("ends", C.POINTER(C.c_uint16)),
                ("accel_depth", C.c_float), ("rgb", C.POINTER(C.c_double))]


class CountersS(C.Structure):
    _fields_ = [("visited", C.c_int64), ("nonempty", C.c_int64), ("tested", C.c_int64),
                ("hits", C.c_int64), ("fragments", C.c_int64)]


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        L.or_grid_setup.restype = C.c_int
        L.or_voxelize.restype = C.c_int
        L.or_paper_record_bytes.restype = C.c_int
        L.or_lod_levels.restype = C.c_int
        L.or_lod.restype = C.c_int
        L.or_cone.restype = C.c_double
        L.or_ao_hemi.restype = C.c_double
        L.or_rep_lines.restype = C.c_int
        L.or_rep_shadow.restype = C.c_int
        L.or_cone.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int32),
                              C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.c_double, C.c_double]
        L.or_ao_grid.restype = C.c_int
        L.or_ao_grid.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int32,
                                 C.c_double, C.c_double, C.POINTER(C.c_double), C.c_int32]
        L.or_shadow_grid.restype = C.c_int
        L.or_shadow_grid.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double), C.c_double,
                                     C.POINTER(C.c_double), C.c_int32]
        L.or_dda.restype = C.c_int64
        L.or_capsule.restype = C.c_int
        L.or_render.restype = C.c_int
        _lib = L
    return _lib


def _grid(grid):
    g = np.asarray(grid if np.ndim(grid) else (grid, grid, grid), dtype=np.int32)
    return np.ascontiguousarray(g)


# ---------------------------------------------------------------------------

def grid_setup(xyz: np.ndarray, grid):
    """float32 [V,3] world vertices -> int32 [V,3] lattice (1/256 voxel)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    g = _grid(grid)
    lat = np.empty(xyz.shape, dtype=np.int32)
    lo = np.zeros(3)
    s = C.c_double()
    rc = lib().or_grid_setup(_p(xyz, C.c_float), C.c_int64(xyz.shape[0]), _p(g, C.c_int32),
                             _p(lat, C.c_int32), _p(lo, C.c_double), C.byref(s))
    if rc != 0:
        raise ValueError("or_grid_setup failed (%d)" % rc)
    return lat, lo, s.value


@dataclass
class OracleCsr:
    offsets: np.ndarray   # uint32 [R^3 + 1]
    records: np.ndarray   # uint64 [S]
    n_events: int
    n_dropped: int
    ends: np.ndarray = None   # uint16 [S] endpoint attributes (per-vertex input), or None


def voxelize(lattice: np.ndarray, curve_off: np.ndarray, attr, grid, bins: int,
             vattr=None) -> OracleCsr:
    """vattr: optional per-vertex attribute bytes (interpolated to the lines'
    endpoints; the records' attribute byte is then their mean)."""
    lat = np.ascontiguousarray(lattice, dtype=np.int32).reshape(-1, 3)
    off = np.ascontiguousarray(curve_off, dtype=np.int64)
    g = _grid(grid)
    n_curves = off.shape[0] - 1
    ap = None
    if attr is not None:
        attr = np.ascontiguousarray(attr, dtype=np.uint8)
        ap = _p(attr, C.c_uint8)
    vp = None
    if vattr is not None:
        vattr = np.ascontiguousarray(vattr, dtype=np.uint8)
        if vattr.shape[0] != lat.shape[0]:
            raise ValueError("vattr needs one byte per vertex")
        vp = _p(vattr, C.c_uint8)
    out = Csr()
    rc = lib().or_voxelize_attr(_p(lat, C.c_int32), _p(off, C.c_int64), ap, vp,
                                C.c_int64(n_curves), _p(g, C.c_int32), C.c_int32(bins),
                                C.byref(out))
    if rc != 0:
        raise ValueError("or_voxelize failed (%d)" % rc)
    try:
        nvox = int(out.n_voxels)
        offs = np.ctypeslib.as_array(out.offsets, shape=(nvox + 1,)).copy()
        n = int(out.n_records)
        recs = (np.ctypeslib.as_array(out.records, shape=(n,)).copy() if n > 0
                else np.zeros(0, dtype=np.uint64))
        ends = None
        if vattr is not None:
            ends = (np.ctypeslib.as_array(out.ends, shape=(n,)).copy() if n > 0
                    else np.zeros(0, dtype=np.uint16))
        return OracleCsr(offs, recs, int(out.n_events), int(out.n_dropped), ends)
    finally:
        lib().or_csr_free(C.byref(out))


def paper_record_bytes(bins: int) -> int:
    return int(lib().or_paper_record_bytes(C.c_int32(bins)))


def lod_levels(grid):
    g = _grid(grid)
    dims = np.zeros((32, 3), dtype=np.int32)
    loff = np.zeros(33, dtype=np.int64)
    n = lib().or_lod_levels(_p(g, C.c_int32), _p(dims, C.c_int32), _p(loff, C.c_int64))
    return dims[:n].copy(), loff[:n + 1].copy()


def lod(csr: OracleCsr, grid, bins: int, lut, opaque: bool):
    """Returns (count, len, rho) flat fp64 pyramids plus (dims, level_off)."""
    g = _grid(grid)
    dims, loff = lod_levels(g)
    total = int(loff[-1])
    cnt = np.zeros(total)
    ln = np.zeros(total)
    rho = np.zeros(total)
    lut = np.ascontiguousarray(lut, dtype=np.float32)
    lib().or_lod(_p(csr.offsets, C.c_uint32), _p(csr.records, C.c_uint64), _p(g, C.c_int32),
                 C.c_int32(bins), _p(lut, C.c_float), C.c_int32(int(opaque)),
                 _p(cnt, C.c_double), _p(ln, C.c_double), _p(rho, C.c_double))
    return cnt, ln, rho, dims, loff


def lod_color(csr: OracleCsr, grid, bins: int, lut, opaque: bool) -> np.ndarray:
    """Colour pyramid [level_off[-1], 3]: sum of length * sigma * lut rgb per
    voxel, averaged up the levels like rho."""
    g = _grid(grid)
    dims, loff = lod_levels(g)
    rgb = np.zeros((int(loff[-1]), 3))
    lut = np.ascontiguousarray(lut, dtype=np.float32)
    lib().or_lod_color(_p(csr.offsets, C.c_uint32), _p(csr.records, C.c_uint64), _p(g, C.c_int32),
                       C.c_int32(bins), _p(lut, C.c_float), C.c_int32(int(opaque)),
                       _p(rgb, C.c_double))
    return rgb


def cone(rho, grid, p, direction, s_max, aperture=1.0) -> float:
    g = _grid(grid)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    d = np.ascontiguousarray(direction, dtype=np.float64)
    return float(lib().or_cone(_p(rho, C.c_double), _p(g, C.c_int32), _p(p, C.c_double),
                               _p(d, C.c_double), C.c_double(s_max), C.c_double(aperture)))


def fibonacci_dirs(n: int) -> np.ndarray:
    d = np.zeros((n, 3))
    lib().or_fibonacci_dirs(C.c_int32(n), _p(d, C.c_double))
    return d


def ao_grid(rho, grid, n_cones=16, radius=15.0, aperture=1.0, threads=0):
    g = _grid(grid)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    ao = np.zeros(int(np.prod(g.astype(np.int64))))
    lib().or_ao_grid(_p(rho, C.c_double), _p(g, C.c_int32), n_cones, radius, aperture,
                     _p(ao, C.c_double), threads)
    return ao


def ao_grid_part(rho, grid, v0, v1, n_cones=16, radius=15.0, aperture=1.0, threads=0):
    """AO of voxels [v0, v1) only (a bounded sample of ao_grid)."""
    g = _grid(grid)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    ao = np.zeros(int(v1 - v0))
    lib().or_ao_grid_part(_p(rho, C.c_double), _p(g, C.c_int32), C.c_int32(n_cones),
                          C.c_double(radius), C.c_double(aperture), C.c_int64(v0), C.c_int64(v1),
                          _p(ao, C.c_double), C.c_int32(threads))
    return ao


def shadow_grid_part(rho, grid, light, v0, v1, aperture=1.0, threads=0):
    """Shadow factors of voxels [v0, v1) only."""
    g = _grid(grid)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    L = np.ascontiguousarray(light, dtype=np.float64)
    sh = np.zeros(int(v1 - v0))
    lib().or_shadow_grid_part(_p(rho, C.c_double), _p(g, C.c_int32), _p(L, C.c_double),
                              C.c_double(aperture), C.c_int64(v0), C.c_int64(v1),
                              _p(sh, C.c_double), C.c_int32(threads))
    return sh


def shadow_grid(rho, grid, light, aperture=1.0, threads=0):
    g = _grid(grid)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    L = np.ascontiguousarray(light, dtype=np.float64)
    sh = np.zeros(int(np.prod(g.astype(np.int64))))
    lib().or_shadow_grid(_p(rho, C.c_double), _p(g, C.c_int32), _p(L, C.c_double),
                         aperture, _p(sh, C.c_double), threads)
    return sh


def rep_lines(csr: OracleCsr, grid, bins: int) -> np.ndarray:
    """Representative line codes (uint32, 0xFFFFFFFF for none), all levels
    flat at lod_levels' offsets."""
    g = _grid(grid)
    dims, loff = lod_levels(g)
    rep = np.zeros(int(loff[-1]), dtype=np.uint32)
    rc = lib().or_rep_lines(_p(csr.offsets, C.c_uint32), _p(csr.records, C.c_uint64),
                            _p(g, C.c_int32), C.c_int32(bins), _p(rep, C.c_uint32))
    if rc < 0:
        raise MemoryError("or_rep_lines")
    return rep


def rep_shadow(rep, grid, bins, level, radius, x, light) -> bool:
    g = _grid(grid)
    rep = np.ascontiguousarray(rep, dtype=np.uint32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    L = np.ascontiguousarray(light, dtype=np.float64)
    return bool(lib().or_rep_shadow(_p(rep, C.c_uint32), _p(g, C.c_int32), C.c_int32(bins),
                                    C.c_int32(level), C.c_double(radius), _p(x, C.c_double),
                                    _p(L, C.c_double)))


def hemi_dirs(n, k: int) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.float64)
    d = np.zeros((k, 3))
    lib().or_hemi_dirs(_p(n, C.c_double), C.c_int32(k), _p(d, C.c_double))
    return d


def ao_hemi(rho, grid, x, n, k=16, radius=15.0) -> float:
    g = _grid(grid)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    return float(lib().or_ao_hemi(_p(rho, C.c_double), _p(g, C.c_int32), _p(x, C.c_double),
                                  _p(n, C.c_double), C.c_int32(k), C.c_double(radius)))


def camera_struct(cam) -> CameraS:
    c = CameraS()
    e, f, r, u = cam.as_arrays()
    c.eye[:] = list(e)
    c.forward[:] = list(f)
    c.right[:] = list(r)
    c.up[:] = list(u)
    c.orthographic = int(cam.orthographic)
    c.width = cam.width
    c.height = cam.height
    return c


def ray(cam, i: int, j: int):
    c = camera_struct(cam)
    o = np.zeros(3, dtype=np.float32)
    d = np.zeros(3, dtype=np.float32)
    lib().or_ray(C.byref(c), C.c_int32(i), C.c_int32(j), _p(o, C.c_float), _p(d, C.c_float))
    return o, d


def dda(grid, o, d, cap: int = 1 << 14):
    g = _grid(grid)
    o = np.ascontiguousarray(o, dtype=np.float32)
    d = np.ascontiguousarray(d, dtype=np.float32)
    cells = np.zeros((cap, 3), dtype=np.int32)
    t0 = np.zeros(cap)
    t1 = np.zeros(cap)
    n = int(lib().or_dda(_p(g, C.c_int32), _p(o, C.c_float), _p(d, C.c_float),
                         _p(cells, C.c_int32), _p(t0, C.c_double), _p(t1, C.c_double),
                         C.c_int64(cap)))
    n = min(n, cap)
    return cells[:n], t0[:n], t1[:n]


def capsule(o, d, a, b, r):
    v = [np.ascontiguousarray(x, dtype=np.float64) for x in (o, d, a, b)]
    ti, to = C.c_double(), C.c_double()
    n = np.zeros(3)
    hit = lib().or_capsule(*[_p(x, C.c_double) for x in v], C.c_double(r), C.byref(ti),
                           C.byref(to), _p(n, C.c_double))
    if not hit:
        return None
    return ti.value, to.value, n


def decode(rec: int, bins: int):
    a = np.zeros(3)
    b = np.zeros(3)
    lib().or_decode(C.c_uint64(int(rec)), C.c_int32(bins), _p(a, C.c_double), _p(b, C.c_double))
    return a, b


def params_struct(radius=0.4, mode=0, opaque=False, alpha_stop=0.95, merge_curves=True,
                  lut=None, shading=1, ka=0.25, kd=0.75, ks=0.2, shininess=16.0,
                  light_dir=(0.0, 0.0, 1.0), distance_alpha=False, ao_mode=0, shadow_mode=0,
                  ao_rays=16, ao_radius=15.0, rep_level=1, accel_depth=0.0):
    p = ParamsS()
    p.radius = radius
    p.mode = mode
    p.opaque = int(opaque)
    p.alpha_stop = alpha_stop
    p.merge_curves = int(merge_curves)
    lut = np.ascontiguousarray(lut, dtype=np.float32)
    p.lut_rgba = _p(lut, C.c_float)
    p.shading = shading
    p.ka, p.kd, p.ks, p.shininess = ka, kd, ks, shininess
    p.light_dir[:] = [float(x) for x in light_dir]
    p.distance_alpha = int(distance_alpha)
    p.ao_mode, p.shadow_mode, p.ao_rays = int(ao_mode), int(shadow_mode), int(ao_rays)
    p.ao_radius, p.rep_level = float(ao_radius), int(rep_level)
    p.accel_depth = float(accel_depth)
    return p, lut  # keep lut alive


def render(csr: OracleCsr, grid, bins: int, cam, pixels=None, ao=None, sh=None,
           threads: int = 0, rho=None, rep=None, rgb=None, **params):
    """fp64 image [H, W, 4] (or [n, 4] for a pixel list) plus counters dict.
    rho (density pyramid) and rep (representative lines) feed the
    per-fragment illumination sources of shading 2."""
    g = _grid(grid)
    c = camera_struct(cam)
    p, keep = params_struct(**params)
    if rho is not None:
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        p.rho = _p(rho, C.c_double)
    if rep is not None:
        rep = np.ascontiguousarray(rep, dtype=np.uint32)
        p.rep = _p(rep, C.c_uint32)
    if rgb is not None:
        rgb = np.ascontiguousarray(rgb, dtype=np.float64)
        p.rgb = _p(rgb, C.c_double)
    ends = getattr(csr, "ends", None)
    if ends is not None:
        ends = np.ascontiguousarray(ends, dtype=np.uint16)
        p.ends = _p(ends, C.c_uint16)
    if pixels is not None:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        n = pix.shape[0]
        pp = _p(pix, C.c_int64)
    else:
        pix = None
        n = cam.width * cam.height
        pp = None
    out = np.zeros((n, 4))
    aop = None
    if ao is not None:
        ao = np.ascontiguousarray(ao, dtype=np.float64)
        aop = _p(ao, C.c_double)
    shp = None
    if sh is not None:
        sh = np.ascontiguousarray(sh, dtype=np.float64)
        shp = _p(sh, C.c_double)
    k = CountersS()
    rc = lib().or_render(_p(csr.offsets, C.c_uint32), _p(csr.records, C.c_uint64),
                         _p(g, C.c_int32), C.c_int32(bins), C.byref(c), C.byref(p), aop, shp,
                         pp, C.c_int64(n), _p(out, C.c_double), C.byref(k), C.c_int32(threads))
    if rc != 0:
        raise ValueError("or_render failed (%d)" % rc)
    del keep
    counters = dict(visited=k.visited, nonempty=k.nonempty, tested=k.tested, hits=k.hits,
                    fragments=k.fragments)
    if pixels is None:
        out = out.reshape(cam.height, cam.width, 4)
    return out, counters
