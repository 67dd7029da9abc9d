"""Python binding of libfassmvs (the MI355X FaSS-MVS hot path).

Argument marshalling only: every step of the pipeline runs in the library's
HIP kernels.  The binding never imports torch: the library owns its HIP
runtime and device memory (``Handle.upload`` / ``DeviceArray``), so no second
HIP runtime shares the process.  Importing raises if the built library is
missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfassmvs.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fassmvs.h")

OK, PENDING = 0, 1
EINVAL, EUNSUPPORTED, ENOMEM, EBUSY, EDEVICE, ENOTFOUND = -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
N_STAGES = 13


class FassmvsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fassmvs status {status}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [
        ("n_levels", C.c_int32), ("census_w", C.c_int32), ("census_h", C.c_int32),
        ("n_paths", C.c_int32), ("sgm_variant", C.c_int32), ("p1", C.c_int32),
        ("p2_mode", C.c_int32), ("p2_fixed", C.c_int32), ("p2_alpha", C.c_double),
        ("p2_beta", C.c_double), ("window_labels", C.c_int32), ("median", C.c_int32),
        ("normal_radius", C.c_int32), ("normal_beta", C.c_double), ("conf_rho_deg", C.c_double),
        ("device", C.c_int32), ("stream", C.c_void_p), ("hbm_budget_bytes", C.c_uint64),
        ("profile", C.c_int32), ("keep_levels", C.c_int32), ("sgm_debug", C.c_int32),
        ("cost", C.c_int32), ("dog_filter", C.c_int32),
    ]


class Image(C.Structure):
    _fields_ = [("pixels", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("stride", C.c_int32), ("R", C.c_double * 9), ("t", C.c_double * 3)]


class ServerResult(C.Structure):
    _fields_ = [("request_id", C.c_uint64), ("stream_id", C.c_int32), ("status", C.c_int32), ("width", C.c_int32),
                ("height", C.c_int32), ("keyframe", C.c_int32), ("n_views", C.c_int32), ("latency_ms", C.c_double)]


class PlaneFamily(C.Structure):
    _fields_ = [("n", C.c_double * 3), ("delta_min", C.c_double), ("delta_max", C.c_double),
                ("count", C.c_int32), ("delta", C.c_void_p), ("depth_min", C.c_double), ("depth_max", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python paper_2112_00821_amd/build.py")
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _declare(L):
    vp, i32, u64, dbl, sz = C.c_void_p, C.c_int32, C.c_uint64, C.c_double, C.c_size_t
    st = C.c_int32
    sigs = {
        "fassmvs_config_default": (None, [vp]),
        "fassmvs_create": (st, [vp, vp]),
        "fassmvs_submit_frame": (st, [vp, vp, vp, vp, i32, vp, vp, i32, i32, vp]),
        "fassmvs_poll": (st, [vp, u64, vp, vp, vp, i32, i32]),
        "fassmvs_submit_batch": (st, [vp, vp, i32, i32, vp]),
        "fassmvs_submit_frame_range": (st, [vp, vp, vp, vp, i32, vp, dbl, dbl, vp, i32, i32, vp]),
        "fassmvs_poll_batch": (st, [vp, u64, i32, vp, vp, vp, i32, i32]),
        "fassmvs_batch_tuning": (st, [vp, vp, vp, vp, vp, vp]),
        "fassmvs_destroy": (None, [vp]),
        "fassmvs_last_error": (C.c_char_p, [vp]),
        "fassmvs_stage_times": (st, [vp, vp, vp, i32]),
        "fassmvs_reset_stage_times": (st, [vp]),
        "fassmvs_stage_name": (C.c_char_p, [i32]),
        "fassmvs_stage_times_level": (st, [vp, i32, vp, vp, i32]),
        "fassmvs_frame_timeline": (st, [vp, vp, i32, vp]),
        "fassmvs_frame_work": (st, [vp, vp, i32]),
        "fassmvs_level_map": (st, [vp, i32, i32, vp, sz]),
        "fassmvs_device_alloc": (st, [vp, sz, vp]),
        "fassmvs_device_free": (st, [vp, vp]),
        "fassmvs_memcpy": (st, [vp, vp, vp, sz, i32]),
        "fassmvs_fill": (st, [vp, vp, C.c_uint8, sz]),
        "fassmvs_synchronize": (st, [vp]),
        "fassmvs_stage_pyr_down": (st, [vp, vp, i32, i32, vp]),
        "fassmvs_stage_census": (st, [vp, vp, i32, i32, i32, i32, vp]),
        "fassmvs_stage_warp": (st, [vp, vp, i32, i32, vp, i32, i32, vp]),
        "fassmvs_stage_cost": (st, [vp, i32, i32, vp, i32, vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]),
        "fassmvs_stage_cost_ncc": (st, [vp, i32, i32, vp, i32, vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]),
        "fassmvs_filter_dog": (st, [vp, vp, i32, i32, vp, vp, vp, vp]),
        "fassmvs_filter_dog_noalloc": (st, [vp, vp, i32, i32, vp, vp, vp, vp]),
        "fassmvs_bounding_planes": (st, [vp, i32, i32, vp, dbl, dbl, vp]),
        "fassmvs_frame_footprint": (st, [vp, i32, i32, i32, vp, i32, vp]),
        "fassmvs_server_create": (st, [vp, i32, u64, vp]),
        "fassmvs_server_open_stream": (st, [vp, vp, i32, i32, vp, i32, i32, dbl, vp]),
        "fassmvs_server_submit": (st, [vp, i32, vp, i32, vp, vp, vp]),
        "fassmvs_server_next": (st, [vp, i32, vp]),
        "fassmvs_server_fetch": (st, [vp, u64, vp, vp, vp, i32]),
        "fassmvs_server_close_stream": (st, [vp, i32]),
        "fassmvs_server_last_error": (C.c_char_p, [vp]),
        "fassmvs_server_destroy": (None, [vp]),
        "fassmvs_cross_ratio_planes": (st, [vp, i32, i32, vp, vp, vp, dbl, dbl, i32, vp, vp]),
        "fassmvs_filter_geometric": (st, [vp, i32, i32, vp, vp, vp, vp, i32, vp, vp, vp, dbl, i32, vp, vp]),
        "fassmvs_stage_sgm": (st, [vp, i32, i32, i32, vp, vp, vp, vp, vp, i32, vp, i32, vp, vp, vp, vp]),
        "fassmvs_stage_sgm_pg": (st, [vp, i32, i32, i32, vp, vp, vp, vp, vp, i32, vp, i32, vp, vp, vp, vp, vp, vp,
                                      vp, vp]),
        "fassmvs_stage_refine": (st, [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "fassmvs_stage_median": (st, [vp, vp, i32, i32, vp]),
        "fassmvs_stage_normals": (st, [vp, vp, vp, i32, i32, vp, i32, dbl, vp, vp, i32, vp, dbl, vp, vp, vp]),
        "fassmvs_stage_seed": (st, [vp, vp, vp, i32, i32, i32, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp,
                                    vp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def exported_symbols_in_header():
    """Every function the public header declares."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fassmvs_[a-z0-9_]+)\s*\(", txt)))


def _arr(a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    return a, a.ctypes.data_as(C.c_void_p)


def default_config(**kw) -> Config:
    c = Config()
    lib().fassmvs_config_default(C.byref(c))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


def config_from_params(params: dict, **kw) -> Config:
    keys = ("n_levels", "census_w", "census_h", "n_paths", "sgm_variant", "p1", "p2_mode", "p2_fixed",
            "p2_alpha", "p2_beta", "window_labels", "median", "normal_radius", "normal_beta", "conf_rho_deg")
    c = default_config()
    for k in keys:
        if k in params:
            setattr(c, k, params[k])
    c.cost = {"census": 0, "ncc": 1}[params.get("cost", "census")]
    c.dog_filter = int(params.get("dog_filter", 0))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def bounding_planes(K, w, h, n, d_min, d_max):
    """(delta_min, delta_max) of the family with normal n for the depth range."""
    Ka, Kp = _arr(K, np.float64)
    na, npp = _arr(n, np.float64)
    out = np.zeros(2)
    st = lib().fassmvs_bounding_planes(Kp, int(w), int(h), npp, float(d_min), float(d_max), out.ctypes.data)
    if st != OK:
        raise FassmvsError(st, "bounding planes: bad input")
    return float(out[0]), float(out[1])


def cross_ratio_planes(K, w, h, R, t, n, delta_min, delta_max, max_planes=4096):
    """Plane distances with one-pixel image steps (delta_max first)."""
    Ka, Kp = _arr(K, np.float64)
    Ra, Rp = _arr(R, np.float64)
    ta, tp = _arr(t, np.float64)
    na, npp = _arr(n, np.float64)
    out = np.zeros(max(max_planes, 1))
    cnt = C.c_int32(0)
    st = lib().fassmvs_cross_ratio_planes(Kp, int(w), int(h), Rp, tp, npp, float(delta_min), float(delta_max),
                                          int(max_planes), out.ctypes.data, C.byref(cnt))
    if st != OK:
        raise FassmvsError(st, f"cross-ratio planes: status {st}, {cnt.value} planes")
    return out[:cnt.value].copy()


def _families(families):
    """ctypes array of plane families from dicts with 'n' and either
    'delta' (an explicit coarsest list), 'delta_min'/'delta_max'/'count', or
    'depth_min'/'depth_max' (bounding planes, delta range left 0).  The
    returned array keeps the explicit lists alive."""
    fams = (PlaneFamily * len(families))()
    keep = []
    for i, f in enumerate(families):
        fams[i].n[:] = [float(x) for x in f["n"]]
        fams[i].delta_min = float(f.get("delta_min", 0.0))
        fams[i].delta_max = float(f.get("delta_max", 0.0))
        fams[i].depth_min = float(f.get("depth_min", 0.0))
        fams[i].depth_max = float(f.get("depth_max", 0.0))
        if f.get("delta") is not None:
            d = np.ascontiguousarray(f["delta"], np.float64)
            keep.append(d)
            fams[i].delta = d.ctypes.data
            fams[i].count = len(d)
        else:
            fams[i].delta = None
            fams[i].count = int(f["count"])
    fams._lists = keep
    return fams


class TimelineEntry(C.Structure):
    _fields_ = [("stage", C.c_int32), ("level", C.c_int32), ("start_ms", C.c_double), ("ms", C.c_double)]


class Frame(C.Structure):
    _fields_ = [("ref", C.c_void_p), ("views", C.c_void_p), ("view_side", C.c_void_p), ("n_views", C.c_int32),
                ("K", C.c_void_p), ("families", C.c_void_p), ("n_families", C.c_int32), ("n_levels", C.c_int32),
                ("window_labels", C.c_int32)]


class Server:
    """Served form: concurrent pipeline slots over several streams (see the
    fassmvs_server_* calls of the header)."""

    def __init__(self, cfg=None, n_slots=4, hbm_budget_bytes=0):
        self.s = C.c_void_p()
        cfg = cfg if cfg is not None else default_config()
        st = lib().fassmvs_server_create(C.byref(cfg), int(n_slots), int(hbm_budget_bytes), C.byref(self.s))
        if st != OK:
            raise FassmvsError(st, lib().fassmvs_last_error(None).decode())
        self.streams = {}

    def _check(self, st):
        if st < 0:
            raise FassmvsError(st, lib().fassmvs_server_last_error(self.s).decode())
        return st

    def open_stream(self, K, width, height, families, max_keyframes=4, min_baseline=1.0):
        sid = C.c_int32()
        Kc = (C.c_double * 9)(*[float(x) for x in np.asarray(K, np.float64).ravel()])
        fams = _families(families)
        self._check(lib().fassmvs_server_open_stream(self.s, Kc, int(width), int(height), fams, len(families),
                                                     int(max_keyframes), float(min_baseline), C.byref(sid)))
        self.streams[sid.value] = (int(width), int(height))
        return sid.value

    def submit(self, stream_id, img, R, t):
        a = np.ascontiguousarray(img, np.uint8)
        rid = C.c_uint64()
        Rc = (C.c_double * 9)(*[float(x) for x in np.asarray(R, np.float64).ravel()])
        tc = (C.c_double * 3)(*[float(x) for x in np.asarray(t, np.float64).ravel()])
        self._check(lib().fassmvs_server_submit(self.s, int(stream_id), a.ctypes.data, a.shape[1], Rc, tc,
                                                C.byref(rid)))
        return rid.value

    def next(self, wait_ms=-1):
        r = ServerResult()
        st = self._check(lib().fassmvs_server_next(self.s, int(wait_ms), C.byref(r)))
        if st == PENDING:
            return None
        return dict(request_id=r.request_id, stream_id=r.stream_id, status=r.status, width=r.width,
                    height=r.height, keyframe=r.keyframe, n_views=r.n_views, latency_ms=r.latency_ms)

    def fetch(self, request_id, w, h):
        depth = np.zeros((h, w), np.float32)
        normal = np.zeros((h, w, 3), np.float32)
        conf = np.zeros((h, w), np.float32)
        self._check(lib().fassmvs_server_fetch(self.s, int(request_id), depth.ctypes.data, normal.ctypes.data,
                                               conf.ctypes.data, MEM_HOST))
        return dict(depth=depth, normal=normal, conf=conf)

    def close_stream(self, stream_id):
        self._check(lib().fassmvs_server_close_stream(self.s, int(stream_id)))

    def close(self):
        if self.s:
            lib().fassmvs_server_destroy(self.s)
            self.s = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class DeviceArray:
    """Device buffer owned by a Handle (numpy-shaped view of raw memory)."""

    def __init__(self, handle, shape, dtype):
        self.handle = handle
        self.shape = tuple(int(s) for s in shape)
        self.dtype = np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape, dtype=np.int64)) * self.dtype.itemsize
        p = C.c_void_p()
        handle._check(lib().fassmvs_device_alloc(handle.h, max(self.nbytes, 1), C.byref(p)))
        self.ptr = p.value

    def numpy(self):
        out = np.empty(self.shape, self.dtype)
        if self.nbytes:
            self.handle._check(lib().fassmvs_memcpy(self.handle.h, out.ctypes.data_as(C.c_void_p),
                                                    C.c_void_p(self.ptr), self.nbytes, 1))
        return out

    def copy_from(self, a):
        a = np.ascontiguousarray(a, dtype=self.dtype)
        assert a.nbytes == self.nbytes
        if self.nbytes:
            self.handle._check(lib().fassmvs_memcpy(self.handle.h, C.c_void_p(self.ptr),
                                                    a.ctypes.data_as(C.c_void_p), self.nbytes, 0))
        return self

    def fill(self, value: int):
        self.handle._check(lib().fassmvs_fill(self.handle.h, C.c_void_p(self.ptr), value, self.nbytes))
        return self

    def free(self):
        if self.ptr and self.handle.h:
            lib().fassmvs_device_free(self.handle.h, C.c_void_p(self.ptr))
        self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def vp(self):
        return C.c_void_p(self.ptr)


def _vp(x):
    if x is None:
        return None
    if isinstance(x, DeviceArray):
        return C.c_void_p(x.ptr)
    return C.c_void_p(int(x))


class Handle:
    def __init__(self, config: Config | None = None, **kw):
        cfg = config if config is not None else default_config(**kw)
        if config is not None:
            for k, v in kw.items():
                setattr(cfg, k, v)
        self.cfg = cfg
        h = C.c_void_p()
        st = lib().fassmvs_create(C.byref(cfg), C.byref(h))
        if st != OK:
            raise FassmvsError(st, lib().fassmvs_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().fassmvs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st not in (OK, PENDING):
            raise FassmvsError(st, lib().fassmvs_last_error(self.h).decode())
        return st

    # ---------------------------------------------------------------- memory
    def empty(self, shape, dtype):
        return DeviceArray(self, shape, dtype)

    def upload(self, a, dtype=None):
        a = np.ascontiguousarray(a, dtype=dtype if dtype is not None else a.dtype)
        return DeviceArray(self, a.shape, a.dtype).copy_from(a)

    def synchronize(self):
        self._check(lib().fassmvs_synchronize(self.h))

    # ---------------------------------------------------------------- frames
    @staticmethod
    def _frame_args(ref, views, side, K, families, keep):
        def mk(v):
            im = Image()
            img = v["img"]
            if isinstance(img, DeviceArray):
                hh, ww = img.shape
                im.pixels = img.ptr
            else:
                a = np.ascontiguousarray(img, np.uint8)
                keep.append(a)
                hh, ww = a.shape
                im.pixels = a.ctypes.data
            im.width, im.height, im.stride = ww, hh, ww
            im.R[:] = [float(x) for x in np.asarray(v["R"], np.float64).ravel()]
            im.t[:] = [float(x) for x in np.asarray(v["t"], np.float64).ravel()]
            return im

        r = mk(ref)
        vs = (Image * len(views))(*[mk(v) for v in views])
        sd = (C.c_int8 * len(side))(*side)
        Kc = (C.c_double * 9)(*[float(x) for x in np.asarray(K, np.float64).ravel()])
        fams = _families(families)
        keep += [r, vs, sd, Kc, fams]
        return r, vs, sd, Kc, fams

    def submit_frame(self, ref, views, side, K, families, mem_kind=MEM_HOST):
        """ref / views: dicts with 'img' (numpy uint8 HxW, or DeviceArray with
        mem_kind=MEM_DEVICE), 'R' (3x3), 't' (3).  families: dicts with 'n' and
        'delta_min', 'delta_max', 'count', or an explicit list 'delta', or a
        depth range 'depth_min', 'depth_max' (see _families)."""
        keep = []
        r, vs, sd, Kc, fams = self._frame_args(ref, views, side, K, families, keep)
        t = C.c_uint64()
        self._check(lib().fassmvs_submit_frame(self.h, C.byref(r), vs, sd, len(views), Kc, fams, len(families),
                                               mem_kind, C.byref(t)))
        return t.value

    def submit_frame_range(self, ref, views, side, K, d_min, d_max, families, mem_kind=MEM_HOST):
        """submit_frame with one depth range for the bundle (families without
        a distance range or list take it through their bounding planes)."""
        keep = []
        r, vs, sd, Kc, fams = self._frame_args(ref, views, side, K, families, keep)
        t = C.c_uint64()
        self._check(lib().fassmvs_submit_frame_range(self.h, C.byref(r), vs, sd, len(views), Kc, float(d_min),
                                                     float(d_max), fams, len(families), mem_kind, C.byref(t)))
        return t.value

    def submit_batch(self, workloads, mem_kind=MEM_HOST):
        """Several scenegen-style frames (dicts with ref, views, side, K,
        families and optionally params n_levels / window_labels) as one batch."""
        keep = []
        frames = (Frame * len(workloads))()
        for i, wl in enumerate(workloads):
            r, vs, sd, Kc, fams = self._frame_args(wl["ref"], wl["views"], wl["side"], wl["K"], wl["families"], keep)
            f = frames[i]
            f.ref, f.views, f.view_side, f.K, f.families = (C.addressof(r), C.addressof(vs), C.addressof(sd),
                                                             C.addressof(Kc), C.addressof(fams))
            f.n_views, f.n_families = len(wl["views"]), len(wl["families"])
            prm = wl.get("params", {})
            f.n_levels = int(prm.get("n_levels", 0))
            f.window_labels = int(prm.get("window_labels", -1))
        t = C.c_uint64()
        self._check(lib().fassmvs_submit_batch(self.h, frames, len(workloads), mem_kind, C.byref(t)))
        return t.value

    def poll_batch(self, ticket, index, depth=None, normal=None, conf=None, mem_kind=MEM_HOST, wait_ms=-1):
        return self._check(lib().fassmvs_poll_batch(self.h, ticket, index, _ptr(depth), _ptr(normal), _ptr(conf),
                                                    mem_kind, wait_ms))

    def run_batch(self, workloads):
        """Run frames as one batch; returns host depth/normal/conf per frame."""
        t = self.submit_batch(workloads)
        out = []
        for i, wl in enumerate(workloads):
            h, w = wl["height"], wl["width"]
            m = dict(depth=np.zeros((h, w), np.float32), normal=np.zeros((h, w, 3), np.float32),
                     conf=np.zeros((h, w), np.float32))
            self.poll_batch(t, i, m["depth"], m["normal"], m["conf"])
            out.append(m)
        return out

    def batch_tuning(self):
        rpt, blocks, groups, graph, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        self._check(lib().fassmvs_batch_tuning(self.h, C.byref(rpt), C.byref(blocks), C.byref(groups), C.byref(graph),
                                               C.byref(ms)))
        return dict(rows_per_thread=rpt.value, sweep_blocks=blocks.value, groups=groups.value, graph=bool(graph.value),
                    batch_ms=ms.value)

    def poll(self, ticket, depth=None, normal=None, conf=None, mem_kind=MEM_HOST, wait_ms=-1):
        st = self._check(lib().fassmvs_poll(self.h, ticket, _ptr(depth), _ptr(normal), _ptr(conf),
                                            mem_kind, wait_ms))
        return st

    def run_frame(self, wl):
        """Run a scenegen workload end to end; returns host depth/normal/conf."""
        h, w = wl["height"], wl["width"]
        t = self.submit_frame(wl["ref"], wl["views"], wl["side"], wl["K"], wl["families"])
        depth = np.zeros((h, w), np.float32)
        normal = np.zeros((h, w, 3), np.float32)
        conf = np.zeros((h, w), np.float32)
        self.poll(t, depth, normal, conf)
        return dict(depth=depth, normal=normal, conf=conf)

    def stage_times(self):
        ms = (C.c_double * N_STAGES)()
        n = (C.c_int32 * N_STAGES)()
        self._check(lib().fassmvs_stage_times(self.h, ms, n, N_STAGES))
        return {lib().fassmvs_stage_name(i).decode(): (ms[i], n[i]) for i in range(N_STAGES)}

    def stage_times_level(self, level):
        ms = (C.c_double * N_STAGES)()
        n = (C.c_int32 * N_STAGES)()
        self._check(lib().fassmvs_stage_times_level(self.h, level, ms, n, N_STAGES))
        return {lib().fassmvs_stage_name(i).decode(): (ms[i], n[i]) for i in range(N_STAGES)}

    def frame_timeline(self):
        """The last polled frame's timed steps: (stage, level, start_ms, ms)."""
        n = C.c_int32()
        self._check(lib().fassmvs_frame_timeline(self.h, None, 0, C.byref(n)))
        buf = (TimelineEntry * max(1, n.value))()
        self._check(lib().fassmvs_frame_timeline(self.h, buf, n.value, C.byref(n)))
        return [(lib().fassmvs_stage_name(e.stage).decode(), e.level, e.start_ms, e.ms) for e in buf[:n.value]]

    def reset_stage_times(self):
        self._check(lib().fassmvs_reset_stage_times(self.h))

    def frame_work(self):
        out = (C.c_double * 9)()
        self._check(lib().fassmvs_frame_work(self.h, out, 9))
        return dict(pixel_hyp=out[0], pixel_hyp_views=out[1], sweep_evaluated=out[2], sgm_design_bytes=out[3],
                    pixel_hyp_level=[out[4 + l] for l in range(5)])

    def level_size(self, level):
        buf = (C.c_int32 * 2)()
        self._check(lib().fassmvs_level_map(self.h, level, 8, buf, 8))
        return buf[0], buf[1]

    def level_map(self, level, what, n_fam=1, D=None):
        w, h = self.level_size(level)
        shapes = {0: ((h, w), np.float32), 1: ((h, w), np.float32), 2: ((h, w, 3), np.float32),
                  3: ((h, w), np.float32), 4: ((h, w), np.int32), 5: ((h, w), np.int32),
                  6: ((n_fam, h, w), np.int32), 7: ((8, h, w, n_fam), np.int8)}
        if what == 9:
            shapes[9] = ((h, w, D), np.uint8)
        elif what == 20:
            shapes[20] = ((h, w), np.uint64)
        elif 10 <= what < 20:
            shapes[what] = ((h, w, D), np.uint16)
        elif what >= 30:
            shapes[what] = ((h, w), np.uint8)
        shape, dt = shapes[what]
        d = self.empty(shape, dt)
        self._check(lib().fassmvs_level_map(self.h, level, what, d.vp, d.nbytes))
        return d.numpy()

    # ---------------------------------------------------------------- stages
    def stage_pyr_down(self, src: DeviceArray):
        h, w = src.shape
        out = self.empty((h // 2, w // 2), np.uint8)
        self._check(lib().fassmvs_stage_pyr_down(self.h, src.vp, w, h, out.vp))
        return out

    def stage_census(self, img: DeviceArray, cw, ch):
        h, w = img.shape
        out = self.empty((h, w), np.uint64)
        self._check(lib().fassmvs_stage_census(self.h, img.vp, w, h, cw, ch, out.vp))
        return out

    def stage_warp(self, src: DeviceArray, H, rw, rh):
        sh, sw = src.shape
        out = self.empty((rh, rw), np.float32)
        Hc, Hp = _arr(H, np.float64)
        self._check(lib().fassmvs_stage_warp(self.h, src.vp, sw, sh, Hp, rw, rh, out.vp))
        return out

    def stage_cost(self, ct_ref: DeviceArray, views, side, cw, ch, G, W, H, offs=None, warped=None):
        h, w = ct_ref.shape
        D = int(np.sum(W))
        out = self.empty((h, w, D), np.uint8)
        vptr = (C.c_void_p * len(side))(*[(v.ptr if v is not None else None) for v in (views or [None] * len(side))])
        sd = (C.c_int8 * len(side))(*side)
        Ga, Gp = _arr(G, np.int32)
        Wa, Wp = _arr(W, np.int32)
        Ha, Hp = _arr(H, np.float64)
        self._check(lib().fassmvs_stage_cost(self.h, w, h, ct_ref.vp, len(side), vptr, sd, cw, ch, len(Ga), Gp, Wp,
                                             Hp, _vp(offs), _vp(warped), out.vp))
        return out

    def stage_cost_ncc(self, ref_img: DeviceArray, views, side, cw, ch, G, W, H, offs=None, warped=None):
        h, w = ref_img.shape
        D = int(np.sum(W))
        out = self.empty((h, w, D), np.uint8)
        vptr = (C.c_void_p * len(side))(*[(v.ptr if v is not None else None) for v in (views or [None] * len(side))])
        sd = (C.c_int8 * len(side))(*side)
        Ga, Gp = _arr(G, np.int32)
        Wa, Wp = _arr(W, np.int32)
        Ha, Hp = _arr(H, np.float64)
        self._check(lib().fassmvs_stage_cost_ncc(self.h, w, h, ref_img.vp, len(side), vptr, sd, cw, ch, len(Ga), Gp,
                                                 Wp, Hp, _vp(offs), _vp(warped), out.vp))
        return out

    def filter_dog(self, img: DeviceArray, depth=None, normal=None, conf=None, want_mask=True):
        """DoG texture filter on device maps (modified in place); returns the mask."""
        h, w = img.shape
        mask = self.empty((h, w), np.uint8) if want_mask else None
        self._check(lib().fassmvs_filter_dog(self.h, img.vp, w, h, _vp(depth), _vp(normal), _vp(conf), _vp(mask)))
        return mask

    def filter_dog_noalloc(self, img: DeviceArray, depth=None, normal=None, conf=None, mask=None):
        """The allocation-free DoG filter (its scratch in the library's static
        device array): maps modified in place, the mask written into the
        caller's device array ``mask`` when given."""
        h, w = img.shape
        self._check(lib().fassmvs_filter_dog_noalloc(self.h, img.vp, w, h, _vp(depth), _vp(normal), _vp(conf),
                                                     _vp(mask)))
        return mask

    def filter_geometric(self, K, depth: DeviceArray, nb_depths, R_rel, t_rel, eta_r=10.0, eta_h=3, normal=None,
                         conf=None):
        """Geometric consistency filter; returns (hits, keep) device arrays."""
        h, w = depth.shape
        hits = self.empty((h, w), np.int32)
        keep = self.empty((h, w), np.uint8)
        n = len(nb_depths)
        ptrs = (C.c_void_p * n)(*[d.ptr for d in nb_depths])
        Ka, Kp = _arr(K, np.float64)
        Ra, Rp = _arr(R_rel, np.float64)
        ta, tp = _arr(t_rel, np.float64)
        self._check(lib().fassmvs_filter_geometric(self.h, w, h, Kp, depth.vp, _vp(normal), _vp(conf), n, ptrs, Rp,
                                                   tp, float(eta_r), int(eta_h), hits.vp, keep.vp))
        return hits, keep

    def stage_sgm(self, S: DeviceArray, W, p1, lut, ref: DeviceArray, n_paths, offs=None, dI=None,
                  want_lr=False, want_sbar=False, want_wta=True):
        h, w, D = S.shape
        Wa, Wp = _arr(W, np.int32)
        la, lp = _arr(lut, np.int32)
        Lr = self.empty((n_paths, h, w, D), np.uint16) if want_lr else None
        Sbar = self.empty((h, w, D), np.uint16) if want_sbar else None
        wta = self.empty((h, w), np.uint16) if want_wta else None
        c3 = self.empty((h, w, 3), np.uint16) if want_wta else None
        self._check(lib().fassmvs_stage_sgm(self.h, w, h, len(Wa), Wp, S.vp, _vp(offs), _vp(dI), ref.vp, int(p1), lp,
                                            n_paths, _vp(Lr), _vp(Sbar), _vp(wta), _vp(c3)))
        return dict(Lr=Lr, Sbar=Sbar, wta=wta, c3=c3)

    def stage_sgm_pg(self, S: DeviceArray, W, G, p1, lut, ref: DeviceArray, n_paths, fam_delta, fam_n, Kinv, step,
                     offs=None, want_lr=False, want_sbar=False, want_wta=True):
        h, w, D = S.shape
        Wa, Wp = _arr(W, np.int32)
        Ga, Gp = _arr(G, np.int32)
        la, lp = _arr(lut, np.int32)
        da, dp = _arr(fam_delta, np.float64)
        na, npp = _arr(fam_n, np.float64)
        ka, kp = _arr(Kinv, np.float64)
        sa, sp = _arr(step, np.float64)
        Lr = self.empty((n_paths, h, w, D), np.uint16) if want_lr else None
        Sbar = self.empty((h, w, D), np.uint16) if want_sbar else None
        wta = self.empty((h, w), np.uint16) if want_wta else None
        c3 = self.empty((h, w, 3), np.uint16) if want_wta else None
        self._check(lib().fassmvs_stage_sgm_pg(self.h, w, h, len(Wa), Wp, Gp, S.vp, _vp(offs), ref.vp, int(p1), lp,
                                               n_paths, dp, npp, kp, sp, _vp(Lr), _vp(Sbar), _vp(wta), _vp(c3)))
        return dict(Lr=Lr, Sbar=Sbar, wta=wta, c3=c3)

    def stage_refine(self, wta, c3, W, G, fam_n, fam_delta, Kinv, offs=None):
        h, w = wta.shape
        Wa, Wp = _arr(W, np.int32)
        Ga, Gp = _arr(G, np.int32)
        na, npp = _arr(fam_n, np.float64)
        da, dp = _arr(fam_delta, np.float64)
        ka, kp = _arr(Kinv, np.float64)
        label = self.empty((h, w), np.int32)
        fam = self.empty((h, w), np.int32)
        depth = self.empty((h, w), np.float32)
        self._check(lib().fassmvs_stage_refine(self.h, w, h, len(Wa), Wp, Gp, _vp(offs), wta.vp, c3.vp, npp, dp, kp,
                                               label.vp, fam.vp, depth.vp))
        return label, fam, depth

    def stage_median(self, d: DeviceArray):
        h, w = d.shape
        out = self.empty((h, w), np.float32)
        self._check(lib().fassmvs_stage_median(self.h, d.vp, w, h, out.vp))
        return out

    def stage_normals(self, depth, img, Kinv, radius, beta, label, fam, fam_n, rho_deg):
        h, w = depth.shape
        ka, kp = _arr(Kinv, np.float64)
        na, npp = _arr(fam_n, np.float64)
        nraw = self.empty((h, w, 3), np.float32)
        normal = self.empty((h, w, 3), np.float32)
        conf = self.empty((h, w), np.float32)
        self._check(lib().fassmvs_stage_normals(self.h, depth.vp, img.vp, w, h, kp, radius, beta, label.vp, fam.vp,
                                                len(na), npp, rho_deg, nraw.vp, normal.vp, conf.vp))
        return nraw, normal, conf

    def stage_seed(self, depth_c, normal_c, fw, fh, Kinv, fam_n, deltas, W, want_dI=True):
        """deltas: the fine level's plane list of every family."""
        ch, cw = depth_c.shape
        G = [len(d) for d in deltas]
        F = len(G)
        ka, kp = _arr(Kinv, np.float64)
        na, npp = _arr(fam_n, np.float64)
        da, dp = _arr(np.concatenate([np.asarray(d, np.float64) for d in deltas]), np.float64)
        Ga, Gp = _arr(G, np.int32)
        Wa, Wp = _arr(W, np.int32)
        dbar = self.empty((fh, fw), np.float32)
        nbar = self.empty((fh, fw, 3), np.float32)
        offs = self.empty((F, fh, fw), np.int32)
        dI = self.empty((8, fh, fw, F), np.int8) if want_dI else None
        self._check(lib().fassmvs_stage_seed(self.h, depth_c.vp, normal_c.vp, cw, ch, fw, fh, kp, F, npp, dp, Gp,
                                             Wp, dbar.vp, nbar.vp, offs.vp, _vp(dI)))
        return dbar, nbar, offs, dI


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, DeviceArray):
        return C.c_void_p(a.ptr)
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)
