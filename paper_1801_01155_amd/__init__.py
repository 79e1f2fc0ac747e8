"""Python binding of liblineset (include/lineset.h): argument marshalling only.

Every step of the rendering pipeline runs in the HIP library; this module
converts torch tensors (device memory) and the current HIP stream into the
C-ABI's plain pointers and maps status codes to exceptions. Functions carry
the C names. Loading fails loudly when the library has not been built:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblineset.so")

LS_OK, LS_EINVAL, LS_ENOMEM, LS_EDEVICE, LS_EUNSUPPORTED, LS_EBUSY, LS_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
(EXPORT_OFFSETS, EXPORT_RECORDS, EXPORT_LOD_COUNT, EXPORT_LOD_LEN, EXPORT_LOD_RHO, EXPORT_AO,
 EXPORT_SHADOW, EXPORT_REP_LINES, EXPORT_ENDS, EXPORT_LOD_COLOR) = range(10)


class LinesetError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class VoxelizeDesc(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("lattice", C.c_void_p), ("curve_off", C.c_void_p),
                ("curve_attr", C.c_void_p), ("n_vertices", C.c_int64), ("n_curves", C.c_int64),
                ("on_device", C.c_int32), ("grid", C.c_int32 * 3), ("bins", C.c_int32),
                ("vertex_attr", C.c_void_p)]


class LodDesc(C.Structure):
    _fields_ = [("lut_rgba", C.c_void_p), ("opaque", C.c_int32), ("build_ao", C.c_int32),
                ("ao_cones", C.c_int32), ("ao_radius", C.c_float), ("cone_aperture", C.c_float),
                ("build_shadow", C.c_int32), ("light_dir", C.c_float * 3),
                ("build_rep_lines", C.c_int32), ("build_color", C.c_int32)]


class CameraS(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("forward", C.c_float * 3), ("right", C.c_float * 3),
                ("up", C.c_float * 3), ("orthographic", C.c_int32), ("width", C.c_int32),
                ("height", C.c_int32)]


class RenderParams(C.Structure):
    _fields_ = [("radius", C.c_float), ("mode", C.c_int32), ("opaque", C.c_int32),
                ("alpha_stop", C.c_float), ("merge_curves", C.c_int32), ("lut_rgba", C.c_void_p),
                ("shading", C.c_int32), ("ka", C.c_float), ("kd", C.c_float), ("ks", C.c_float),
                ("shininess", C.c_float), ("light_dir", C.c_float * 3),
                ("distance_alpha", C.c_int32), ("ao_mode", C.c_int32),
                ("shadow_mode", C.c_int32), ("ao_rays", C.c_int32), ("ao_radius", C.c_float),
                ("rep_level", C.c_int32), ("accel_depth", C.c_float)]


class RenderCounters(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("visited", "nonempty", "tested", "hits", "fragments",
                                          "list_bytes", "sort_passes", "merge_evictions",
                                          "macro_skips", "merge_live_evictions",
                                          "merge_overflow_rays")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("grid", C.c_int32 * 3), ("bins", C.c_int32), ("n_curves", C.c_int64),
                ("n_vertices", C.c_int64), ("n_records", C.c_int64),
                ("n_record_slots", C.c_int64), ("nonempty_voxels", C.c_int64),
                ("max_list", C.c_int64), ("n_levels", C.c_int32), ("has_ao", C.c_int32),
                ("has_shadow", C.c_int32), ("has_rep_lines", C.c_int32),
                ("has_vertex_attr", C.c_int32), ("has_color", C.c_int32),
                ("level_dims", (C.c_int32 * 3) * 32),
                ("level_off", C.c_int64 * 33), ("lo_scale", C.c_double * 4),
                ("device_bytes", C.c_size_t)]


_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"liblineset.so not built ({LIB_PATH}); run "
                              "`python -m paper_1801_01155_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.ls_last_error.restype = C.c_char_p
        L.lineset_voxelize.argtypes = [C.POINTER(VoxelizeDesc), C.c_void_p, C.POINTER(C.c_void_p)]
        L.lineset_destroy.argtypes = [C.c_void_p]
        L.lineset_destroy.restype = None
        L.lineset_build_lod.argtypes = [C.c_void_p, C.POINTER(LodDesc), C.c_void_p]
        L.lineset_render.argtypes = [C.c_void_p, C.POINTER(CameraS), C.POINTER(RenderParams),
                                     C.c_void_p, C.c_void_p]
        L.lineset_render_counted.argtypes = [C.c_void_p, C.POINTER(CameraS),
                                             C.POINTER(RenderParams), C.c_void_p,
                                             C.POINTER(RenderCounters), C.c_void_p]
        L.lineset_info.argtypes = [C.c_void_p, C.POINTER(Info)]
        L.lineset_export.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.c_int32,
                                     C.c_void_p]
        L.lineset_grid_setup.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.c_void_p,
                                         C.POINTER(C.c_double), C.c_void_p]
        _lib = L
    return _lib


def _check(rc):
    if rc != LS_OK:
        raise LinesetError(rc, lib().ls_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _empty(shape, dtype, stream=None, device="cuda"):
    """A new device tensor allocated on the stream the library call will use,
    so torch's allocator does not hand its memory to another stream while
    that call may still write it."""
    if stream is None:
        return torch.empty(shape, dtype=dtype, device=device)
    with torch.cuda.stream(stream):
        return torch.empty(shape, dtype=dtype, device=device)


def _dev(t, dtype):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    return t.to(device="cuda", dtype=dtype).contiguous()


def _grid3(grid):
    g = [int(grid)] * 3 if isinstance(grid, int) else [int(x) for x in grid]
    return (C.c_int32 * 3)(*g)


# ---------------------------------------------------------------------------
# C entry points, same names

def lineset_grid_setup(xyz, grid, stream=None):
    """Device float [V,3] -> device int32 [V,3] lattice; returns (lattice, lo_scale)."""
    xyz = _dev(xyz, torch.float32)
    lat = _empty(xyz.shape, torch.int32, stream, xyz.device)
    ls = (C.c_double * 4)()
    _check(lib().lineset_grid_setup(_ptr(xyz), xyz.shape[0], _grid3(grid), _ptr(lat), ls,
                                    _stream(stream)))
    return lat, list(ls)


class LineSet:
    """Owns an ls_lineset_t handle."""

    def __init__(self, handle):
        self.handle = C.c_void_p(handle)

    def __del__(self):
        self.close()

    def close(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.lineset_destroy(self.handle)
        self.handle = None

    def info(self) -> Info:
        return lineset_info(self)


def lineset_voxelize(curve_off, grid, bins=32, xyz=None, lattice=None, attr=None,
                     stream=None, vattr=None) -> LineSet:
    """vattr: optional per-vertex attribute bytes (interpolated to the face
    crossings; the lines keep their endpoint attributes)."""
    d = VoxelizeDesc()
    keep = []
    if xyz is not None:
        xyz = _dev(xyz, torch.float32)
        keep.append(xyz)
        d.xyz = xyz.data_ptr()
        d.n_vertices = xyz.shape[0]
    if lattice is not None:
        lattice = _dev(lattice, torch.int32)
        keep.append(lattice)
        d.lattice = lattice.data_ptr()
        d.n_vertices = lattice.shape[0]
    off = _dev(curve_off, torch.int64)
    keep.append(off)
    d.curve_off = off.data_ptr()
    d.n_curves = off.shape[0] - 1
    if attr is not None:
        attr = _dev(attr, torch.uint8)
        keep.append(attr)
        d.curve_attr = attr.data_ptr()
    if vattr is not None:
        vattr = _dev(vattr, torch.uint8)
        keep.append(vattr)
        d.vertex_attr = vattr.data_ptr()
    d.on_device = 1
    d.grid = _grid3(grid)
    d.bins = bins
    h = C.c_void_p()
    _check(lib().lineset_voxelize(C.byref(d), _stream(stream), C.byref(h)))
    return LineSet(h.value)


class UpdateDesc(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("lattice", C.c_void_p), ("curve_off", C.c_void_p),
                ("curve_attr", C.c_void_p), ("n_vertices", C.c_int64), ("n_curves", C.c_int64),
                ("remove_ids", C.c_void_p), ("n_remove", C.c_int64), ("on_device", C.c_int32)]


def lineset_update(ls: LineSet, remove=None, curve_off=None, xyz=None, lattice=None, attr=None,
                   stream=None) -> None:
    """Removes curves by id and appends curves (device tensors or arrays)."""
    d = UpdateDesc()
    keep = []
    if remove is not None:
        rm = _dev(remove, torch.int64)
        keep.append(rm)
        d.remove_ids = rm.data_ptr() if rm.numel() else None
        d.n_remove = rm.numel()
    if curve_off is not None:
        off = _dev(curve_off, torch.int64)
        keep.append(off)
        d.curve_off = off.data_ptr()
        d.n_curves = off.shape[0] - 1
        for name, arr, dt in (("xyz", xyz, torch.float32), ("lattice", lattice, torch.int32)):
            if arr is not None:
                t = _dev(arr, dt)
                keep.append(t)
                setattr(d, name, t.data_ptr() if t.numel() else None)
                d.n_vertices = t.shape[0]
        if attr is not None:
            a = _dev(attr, torch.uint8)
            keep.append(a)
            d.curve_attr = a.data_ptr() if a.numel() else None
    d.on_device = 1
    L = lib()
    L.lineset_update.argtypes = [C.c_void_p, C.POINTER(UpdateDesc), C.c_void_p]
    _check(L.lineset_update(ls.handle, C.byref(d), _stream(stream)))


def lineset_build_lod(ls: LineSet, lut, opaque=False, build_ao=False, ao_cones=16,
                      ao_radius=15.0, cone_aperture=1.0, build_shadow=False,
                      light_dir=(0.0, 0.0, 1.0), build_rep_lines=False, build_color=False,
                      stream=None):
    lut = _dev(lut, torch.float32)
    d = LodDesc()
    d.lut_rgba = lut.data_ptr()
    d.opaque = int(opaque)
    d.build_ao = int(build_ao)
    d.ao_cones = ao_cones
    d.ao_radius = ao_radius
    d.cone_aperture = cone_aperture
    d.build_shadow = int(build_shadow)
    d.light_dir = (C.c_float * 3)(*light_dir)
    d.build_rep_lines = int(build_rep_lines)
    d.build_color = int(build_color)
    _check(lib().lineset_build_lod(ls.handle, C.byref(d), _stream(stream)))


def camera_struct(cam) -> CameraS:
    c = CameraS()
    c.eye = (C.c_float * 3)(*cam.eye)
    c.forward = (C.c_float * 3)(*cam.forward)
    c.right = (C.c_float * 3)(*cam.right)
    c.up = (C.c_float * 3)(*cam.up)
    c.orthographic = int(cam.orthographic)
    c.width = cam.width
    c.height = cam.height
    return c


def render_params(lut, radius=0.4, mode=0, opaque=False, alpha_stop=0.95, merge_curves=True,
                  shading=1, ka=0.25, kd=0.75, ks=0.2, shininess=16.0,
                  light_dir=(0.0, 0.0, 1.0), distance_alpha=False, ao_mode=0, shadow_mode=0,
                  ao_rays=16, ao_radius=15.0, rep_level=1, accel_depth=0.0) -> RenderParams:
    p = RenderParams()
    p.radius = radius
    p.mode = mode
    p.opaque = int(opaque)
    p.alpha_stop = alpha_stop
    p.merge_curves = int(merge_curves)
    p.lut_rgba = lut.data_ptr()
    p.shading = shading
    p.ka, p.kd, p.ks, p.shininess = ka, kd, ks, shininess
    p.light_dir = (C.c_float * 3)(*light_dir)
    p.distance_alpha = int(distance_alpha)
    p.ao_mode, p.shadow_mode, p.ao_rays = int(ao_mode), int(shadow_mode), int(ao_rays)
    p.ao_radius, p.rep_level = float(ao_radius), int(rep_level)
    p.accel_depth = float(accel_depth)
    return p


def lineset_render(ls: LineSet, cam, lut, out=None, stream=None, **params):
    """Renders into a device float tensor [H, W, 4] (premultiplied RGBA)."""
    lut = _dev(lut, torch.float32)
    if out is None:
        out = _empty((cam.height, cam.width, 4), torch.float32, stream)
    c = camera_struct(cam)
    p = render_params(lut, **params)
    _check(lib().lineset_render(ls.handle, C.byref(c), C.byref(p), _ptr(out), _stream(stream)))
    return out


def lineset_render_counted(ls: LineSet, cam, lut, out=None, stream=None, **params):
    lut = _dev(lut, torch.float32)
    if out is None:
        out = _empty((cam.height, cam.width, 4), torch.float32, stream)
    c = camera_struct(cam)
    p = render_params(lut, **params)
    k = RenderCounters()
    _check(lib().lineset_render_counted(ls.handle, C.byref(c), C.byref(p), _ptr(out),
                                        C.byref(k), _stream(stream)))
    return out, k.as_dict()


def lineset_render_limits() -> dict:
    """Compile-time limits of the ray caster ({'merge_slots'})."""
    m = C.c_int32()
    _check(lib().lineset_render_limits(C.byref(m)))
    return {"merge_slots": m.value}


def lineset_info(ls: LineSet) -> Info:
    i = Info()
    _check(lib().lineset_info(ls.handle, C.byref(i)))
    return i


def lineset_pool_trim() -> None:
    """Frees the device memory cache's unused blocks (all devices)."""
    L = lib()
    L.lineset_pool_trim.restype = None
    L.lineset_pool_trim()


def lineset_pool_stats(device: int = 0) -> dict:
    """{'cached_bytes', 'held_bytes'} of the device memory cache on `device`."""
    c, h = C.c_size_t(0), C.c_size_t(0)
    L = lib()
    L.lineset_pool_stats.argtypes = [C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    _check(L.lineset_pool_stats(C.c_int32(device), C.byref(c), C.byref(h)))
    return {"cached_bytes": c.value, "held_bytes": h.value}


_EXPORT_DTYPE = {EXPORT_OFFSETS: torch.int32, EXPORT_RECORDS: torch.int64,
                 EXPORT_LOD_COUNT: torch.float32, EXPORT_LOD_LEN: torch.float32,
                 EXPORT_LOD_RHO: torch.float32, EXPORT_AO: torch.float32,
                 EXPORT_SHADOW: torch.float32, EXPORT_REP_LINES: torch.int32,
                 EXPORT_ENDS: torch.int16, EXPORT_LOD_COLOR: torch.float32}


def lineset_export(ls: LineSet, what: int, stream=None) -> torch.Tensor:
    """Copies a buffer of the set into a new device tensor (offsets as int32
    bit patterns of uint32, records as int64 bit patterns of uint64)."""
    i = lineset_info(ls)
    nvox = i.grid[0] * i.grid[1] * i.grid[2]
    n = {EXPORT_OFFSETS: nvox + 1, EXPORT_RECORDS: i.n_records,
         EXPORT_LOD_COUNT: i.level_off[i.n_levels] if i.n_levels else 0,
         EXPORT_LOD_LEN: i.level_off[i.n_levels] if i.n_levels else 0,
         EXPORT_LOD_RHO: i.level_off[i.n_levels] if i.n_levels else 0,
         EXPORT_AO: nvox, EXPORT_SHADOW: nvox,
         EXPORT_REP_LINES: i.level_off[i.n_levels] if i.has_rep_lines else 0,
         EXPORT_ENDS: i.n_records if i.has_vertex_attr else 0,
         EXPORT_LOD_COLOR: 3 * i.level_off[i.n_levels] if i.has_color else 0}[what]
    t = _empty(max(int(n), 1), _EXPORT_DTYPE[what], stream)
    _check(lib().lineset_export(ls.handle, what, _ptr(t), t.numel() * t.element_size(), 1,
                                _stream(stream)))
    return t[:n]


# ---------------------------------------------------------------------------
# Batched rendering

BATCH_AUTOTUNE, BATCH_GRAPH = 1, 2


class ViewS(C.Structure):
    _fields_ = [("set", C.c_void_p), ("cam", CameraS), ("params", RenderParams),
                ("rgba_out", C.c_void_p)]


class BatchConfig(C.Structure):
    _fields_ = [("waves_x", C.c_int32), ("waves_y", C.c_int32), ("blocks", C.c_int32),
                ("n_tiles", C.c_int32), ("autotuned", C.c_int32), ("candidates", C.c_int32),
                ("tuned_ms", C.c_float), ("graph", C.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def _bind_batch(L):
    if getattr(L, "_batch_bound", False):
        return
    L.lineset_batch_create.argtypes = [C.POINTER(ViewS), C.c_int32, C.c_int32, C.c_void_p,
                                       C.POINTER(C.c_void_p)]
    L.lineset_batch_create_plan.argtypes = [C.POINTER(ViewS), C.c_int32, C.c_int32, C.c_int32,
                                            C.c_int32, C.c_int32, C.c_void_p,
                                            C.POINTER(C.c_void_p)]
    L.lineset_batch_candidates.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int32), C.c_int32,
                                           C.POINTER(C.c_int32)]
    L.lineset_batch_render.argtypes = [C.c_void_p, C.c_void_p]
    L.lineset_batch_render_counted.argtypes = [C.c_void_p, C.POINTER(RenderCounters), C.c_void_p]
    L.lineset_batch_config.argtypes = [C.c_void_p, C.POINTER(BatchConfig)]
    L.lineset_batch_destroy.argtypes = [C.c_void_p]
    L.lineset_batch_destroy.restype = None
    L.lineset_render_batch.argtypes = [C.POINTER(ViewS), C.c_int32, C.c_void_p]
    L.lineset_render_batch_static.argtypes = [C.POINTER(ViewS), C.c_int32, C.c_void_p]
    L._batch_bound = True


def make_views(items):
    """items: sequence of (LineSet, camera, lut_tensor, out_tensor, params dict)."""
    arr = (ViewS * len(items))()
    for k, (ls, cam, lut, out, params) in enumerate(items):
        arr[k].set = ls.handle.value
        arr[k].cam = camera_struct(cam)
        arr[k].params = render_params(lut, **params)
        arr[k].rgba_out = out.data_ptr()
    return arr


class Batch:
    """Owns an ls_batch_t (one persistent launch over many views)."""

    def __init__(self, items, autotune=False, graph=False, stream=None, plan=None):
        """plan: (waves_x, waves_y, grid_mult) to fix the plan (one of
        batch_candidates()) instead of the cache / autotuner / default."""
        L = lib()
        _bind_batch(L)
        self._items = list(items)      # keep sets, LUTs and outputs alive
        self._views = make_views(self._items)
        flags = (BATCH_AUTOTUNE if autotune else 0) | (BATCH_GRAPH if graph else 0)
        h = C.c_void_p()
        if plan is None:
            _check(L.lineset_batch_create(self._views, len(self._items), flags, _stream(stream),
                                          C.byref(h)))
        else:
            wx, wy, m = plan
            _check(L.lineset_batch_create_plan(self._views, len(self._items), wx, wy, m, flags,
                                               _stream(stream), C.byref(h)))
        self.handle = h

    def render(self, stream=None):
        _check(lib().lineset_batch_render(self.handle, _stream(stream)))

    def render_counted(self, stream=None):
        k = RenderCounters()
        _check(lib().lineset_batch_render_counted(self.handle, C.byref(k), _stream(stream)))
        return k.as_dict()

    def config(self):
        c = BatchConfig()
        _check(lib().lineset_batch_config(self.handle, C.byref(c)))
        return c.as_dict()

    def close(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.lineset_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()


def batch_candidates():
    """The autotuner's plans [(waves_x, waves_y, grid_mult), ...] in its order."""
    L = lib()
    _bind_batch(L)
    n = C.c_int32()
    _check(L.lineset_batch_candidates(None, None, None, 0, C.byref(n)))
    wx, wy, m = (C.c_int32 * n.value)(), (C.c_int32 * n.value)(), (C.c_int32 * n.value)()
    _check(L.lineset_batch_candidates(wx, wy, m, n.value, C.byref(n)))
    return [(wx[k], wy[k], m[k]) for k in range(n.value)]


def lineset_render_batch(items, stream=None):
    L = lib()
    _bind_batch(L)
    views = make_views(items)
    _check(L.lineset_render_batch(views, len(items), _stream(stream)))


def lineset_render_batch_static(items, stream=None):
    """lineset_render_batch without device allocation (library-owned fixed
    scratch, at most 256 views)."""
    L = lib()
    _bind_batch(L)
    views = make_views(items)
    _check(L.lineset_render_batch_static(views, len(items), _stream(stream)))


# ---------------------------------------------------------------------------
# Render server

class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("n_slots", C.c_int32),
                ("max_batch_views", C.c_int32), ("max_queue", C.c_int32),
                ("output_arena_bytes", C.c_size_t)]


class ServerReport(C.Structure):
    _fields_ = [("completed", C.c_int64), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("max_ms", C.c_double), ("mrays_per_s", C.c_double), ("batches", C.c_int64),
                ("mean_batch", C.c_double), ("queued", C.c_int64), ("max_queue_depth", C.c_int64),
                ("rejected", C.c_int64), ("resident_bytes", C.c_size_t),
                ("inflight_bytes", C.c_size_t), ("held_for_memory", C.c_int64),
                ("arena_bytes", C.c_size_t), ("arena_in_use", C.c_size_t)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def _bind_server(L):
    if getattr(L, "_server_bound", False):
        return
    L.ls_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]
    L.ls_server_add_lineset.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]
    L.ls_server_submit.argtypes = [C.c_void_p, C.c_int32, C.POINTER(CameraS),
                                   C.POINTER(RenderParams), C.c_void_p, C.c_void_p,
                                   C.POINTER(C.c_uint64)]
    L.ls_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_int64]
    L.ls_server_result.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_size_t, C.c_int32,
                                   C.c_void_p]
    L.ls_server_stats.argtypes = [C.c_void_p, C.POINTER(ServerReport)]
    L.ls_server_destroy.argtypes = [C.c_void_p]
    L.ls_server_destroy.restype = None
    L._server_bound = True


class Server:
    """Owns an ls_server_t. Keeps the sets, LUTs and outputs of pending
    requests alive until they are waited for."""

    def __init__(self, hbm_budget_bytes, n_slots=2, max_batch_views=64, max_queue=4096,
                 output_arena_bytes=0):
        L = lib()
        _bind_server(L)
        cfg = ServerConfig(hbm_budget_bytes, n_slots, max_batch_views, max_queue,
                           output_arena_bytes)
        h = C.c_void_p()
        _check(L.ls_server_create(C.byref(cfg), C.byref(h)))
        self.handle = h
        self._sets = []
        self._pending = {}

    def add_lineset(self, ls: LineSet) -> int:
        sid = C.c_int32()
        _check(lib().ls_server_add_lineset(self.handle, ls.handle, C.byref(sid)))
        self._sets.append(ls)
        return sid.value

    def submit(self, set_id, cam, lut, out=None, stream=None, **params) -> int:
        """Queues a render into `out` (device tensor [H, W, 4]), or into the
        server's output arena when `out` is None (collect it with result()).
        Work queued on `stream` (default: the current stream) before the call
        is done before the render."""
        c = camera_struct(cam)
        p = render_params(lut, **params)
        t = C.c_uint64()
        _check(lib().ls_server_submit(self.handle, set_id, C.byref(c), C.byref(p),
                                      _ptr(out), _stream(stream), C.byref(t)))
        self._pending[t.value] = (lut, out)
        return t.value

    def result(self, ticket, out, stream=None):
        """Copies a completed arena request's image into `out` (device tensor
        [H, W, 4]) and returns its arena block."""
        _check(lib().ls_server_result(self.handle, C.c_uint64(ticket), _ptr(out),
                                      out.numel() * out.element_size(), 1, _stream(stream)))
        self._pending.pop(ticket, None)
        return out

    def wait(self, ticket, timeout_us=-1):
        rc = lib().ls_server_wait(self.handle, C.c_uint64(ticket), C.c_int64(timeout_us))
        if rc == LS_ETIMEOUT:
            return False
        _check(rc)
        if self._pending.get(ticket, (None, None))[1] is not None:
            self._pending.pop(ticket, None)
        return True

    def stats(self):
        r = ServerReport()
        _check(lib().ls_server_stats(self.handle, C.byref(r)))
        return r.as_dict()

    def close(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.ls_server_destroy(self.handle)
        self.handle = None
        self._pending = {}

    def __del__(self):
        self.close()
