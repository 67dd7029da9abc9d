"""FaSS-MVS CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain single-threaded reference of the method's hot path, used by the tests,
the smoke check and the benchmark's CPU-baseline leg only.  The per-pixel
stages live in ``fassmvs_oracle.cpp`` (built to ``liboracle.so``); this
module binds them with ctypes and drives one frame coarse-to-fine
(pipeline overview of the paper's methodology section).  It shares no code
with the GPU library.

Parity status: pinned by the CPU tests (closed forms, brute force, library
routines on special cases, invariants, ground-truth recovery); the normal
smoothing through fixed points, a two-pixel weight ratio and, on flat
intensity, a Gaussian correlation; the confidence through closed forms.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fassmvs_oracle.cpp")
# FASSMVS_ORACLE_SANITIZE=1: an AddressSanitizer + UndefinedBehaviorSanitizer
# build (the process must preload the ASan runtime; see
# tests/test_sanitizers.py)
_SANITIZE = os.environ.get("FASSMVS_ORACLE_SANITIZE", "0") not in ("", "0")
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=undefined"]

DIRS = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (no fused multiply-add, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        opt = _SAN_FLAGS if _SANITIZE else ["-O2"]
        subprocess.check_call(["g++", *opt, "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _declare(L):
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    sig = {
        "or_kinv_level": (i, [vp, i, vp, vp]),
        "or_relative_pose": (None, [vp, vp, vp, vp, vp, vp]),
        "or_homography": (None, [vp, vp, vp, vp, vp, d, vp]),
        "or_plane_list": (None, [d, d, i, vp]),
        "or_depth_on_plane": (d, [vp, vp, d, i, i]),
        "or_p2_lut": (None, [i, i, i, d, d, vp]),
        "or_pyr_down": (i, [vp, i, i, vp]),
        "or_warp": (None, [vp, i, i, vp, i, i, vp]),
        "or_census": (i, [vp, i, i, i, i, vp]),
        "or_census_u8": (i, [vp, i, i, i, i, vp]),
        "or_cost_volume": (i, [i, i, vp, i, vp, vp, i, i, i, vp, vp, vp, vp, vp]),
        "or_cost_sample": (i, [i, i, vp, i, vp, vp, i, i, i, vp, vp, i, i, i, i]),
        "or_cost_pixels": (i, [i, i, vp, i, vp, vp, i, i, i, vp, vp, vp, vp, i, vp, vp]),
        "or_ncc_cost_volume": (i, [i, i, vp, i, vp, vp, i, i, i, vp, vp, vp, vp, vp]),
        "or_ncc_cost_pixels": (i, [i, i, vp, i, vp, vp, i, i, i, vp, vp, vp, vp, i, vp, vp]),
        "or_ncc_window": (i, [vp, vp, i, i]),
        "or_sgm": (i, [i, i, i, vp, vp, vp, vp, i, vp, vp, i, vp, vp]),
        "or_sgm_pg": (i, [i, i, i, vp, vp, vp, vp, i, vp, vp, i, vp, vp, i, vp, vp, vp, vp, vp]),
        "or_wta_refine": (None, [i, i, i, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "or_median5": (None, [vp, i, i, vp]),
        "or_normals": (None, [vp, i, i, vp, vp]),
        "or_normal_smooth": (None, [vp, vp, i, i, i, d, vp]),
        "or_confidence": (None, [vp, vp, vp, vp, i, i, d, vp]),
        "or_upsample_nn": (None, [vp, i, i, i, i, i, vp]),
        "or_window_offsets": (None, [vp, i, i, vp, i, vp, vp, vp, vp, vp]),
        "or_delta_i": (None, [vp, vp, i, i, vp, i, vp, vp, vp, vp]),
        "or_level_list": (i, [vp, i, i, vp]),
        "or_list_index": (d, [vp, i, d]),
        "or_gauss_taps": (None, [d, i, vp]),
        "or_dog": (None, [vp, i, i, d, i, vp]),
        "or_dog_mask": (None, [vp, i, i, d, i, d, i, i, vp]),
        "or_speckle": (None, [vp, i, i, i, i]),
        "or_geo_consistency": (None, [i, i, vp, vp, i, vp, vp, vp, d, i, vp, vp]),
        "or_bounding_planes": (i, [vp, i, i, vp, d, d, vp]),
        "or_cross_ratio_planes": (i, [vp, i, i, vp, vp, vp, d, d, i, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# thin wrappers
# ---------------------------------------------------------------------------

def kinv_level(K, level):
    K = _c(K, np.float64)
    Ki = np.zeros(9)
    Kl = np.zeros(9)
    if lib().or_kinv_level(_p(K), level, _p(Ki), _p(Kl)) != 0:
        raise ValueError("intrinsics must be upper triangular with K[2,2] = 1")
    return Ki.reshape(3, 3), Kl.reshape(3, 3)


def relative_pose(Rref, tref, Rk, tk):
    R = np.zeros(9)
    t = np.zeros(3)
    lib().or_relative_pose(_p(_c(Rref, np.float64)), _p(_c(tref, np.float64)),
                           _p(_c(Rk, np.float64)), _p(_c(tk, np.float64)), _p(R), _p(t))
    return R.reshape(3, 3), t


def homography(Kl, Kinv, R, t, n, delta):
    H = np.zeros(9)
    lib().or_homography(_p(_c(Kl, np.float64)), _p(_c(Kinv, np.float64)), _p(_c(R, np.float64)),
                        _p(_c(t, np.float64)), _p(_c(n, np.float64)), float(delta), _p(H))
    return H.reshape(3, 3)


def plane_list(dmin, dmax, G):
    out = np.zeros(G)
    lib().or_plane_list(float(dmin), float(dmax), int(G), _p(out))
    return out


def level_list(top, G):
    """The G-plane list of a finer level from the coarsest list ``top``
    (increasing distances): inverse distance interpolated at the fractional
    indices j (len(top) - 1) / (G - 1)."""
    top = _c(top, np.float64)
    out = np.zeros(int(G))
    if lib().or_level_list(_p(top), len(top), int(G), _p(out)) != 0:
        raise ValueError("level_list: lists need at least two planes")
    return out


def list_index(deltas, inv_delta):
    """Continuous index of an inverse distance in a plane list (piecewise
    linear between the planes, end intervals extended)."""
    d = _c(deltas, np.float64)
    return lib().or_list_index(_p(d), len(d), float(inv_delta))


def depth_on_plane(Kinv, n, delta, x, y):
    return lib().or_depth_on_plane(_p(_c(Kinv, np.float64)), _p(_c(n, np.float64)), float(delta), int(x), int(y))


def p2_lut(p1, mode, p2_fixed, alpha, beta):
    lut = np.zeros(256, np.int32)
    lib().or_p2_lut(int(p1), int(mode), int(p2_fixed), float(alpha), float(beta), _p(lut))
    return lut


def pyr_down(img):
    img = _c(img, np.uint8)
    h, w = img.shape
    out = np.zeros((h // 2, w // 2), np.uint8)
    if lib().or_pyr_down(_p(img), w, h, _p(out)) != 0:
        raise ValueError("image too small to downsample")
    return out


def warp(src, H, rw, rh):
    src = _c(src, np.uint8)
    out = np.zeros((rh, rw), np.float32)
    lib().or_warp(_p(src), src.shape[1], src.shape[0], _p(_c(H, np.float64)), rw, rh, _p(out))
    return out


def census(img, cw, ch):
    h, w = img.shape
    out = np.zeros((h, w), np.uint64)
    if img.dtype == np.uint8:
        r = lib().or_census_u8(_p(_c(img, np.uint8)), w, h, cw, ch, _p(out))
    else:
        r = lib().or_census(_p(_c(img, np.float32)), w, h, cw, ch, _p(out))
    if r != 0:
        raise ValueError("census window must be odd and at most 65 pixels")
    return out


def _view_ptrs(views):
    arrs = [_c(v, np.uint8) for v in views]
    ptrs = (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    return arrs, ptrs


def cost_volume(ct_ref, views, side, cw, ch, G, W, H, offs=None):
    """S[h][w][sum W] uint8; H: [n_views][sum G][3][3]."""
    h, w = ct_ref.shape
    G = np.asarray(G, np.int32)
    W = np.asarray(W, np.int32)
    arrs, ptrs = _view_ptrs(views)
    side = _c(side, np.int8)
    H = _c(H, np.float64)
    S = np.zeros((h, w, int(W.sum())), np.uint8)
    offs_c = _c(offs, np.int32) if offs is not None else None
    r = lib().or_cost_volume(w, h, _p(_c(ct_ref, np.uint64)), len(arrs), C.cast(ptrs, C.c_void_p), _p(side),
                             cw, ch, len(G), _p(G), _p(W), _p(H), _p(offs_c), _p(S))
    if r != 0:
        raise ValueError("cost volume: bad arguments or 8-bit overflow (%d)" % r)
    return S


def ncc_cost_volume(ref_img, views, side, cw, ch, G, W, H, offs=None):
    """NCC cost volume S[h][w][sum W] uint8 (negated, truncated, scaled NCC;
    mean over each subset); H: [n_views][sum G][3][3]."""
    ref_img = _c(ref_img, np.uint8)
    h, w = ref_img.shape
    G = np.asarray(G, np.int32)
    W = np.asarray(W, np.int32)
    arrs, ptrs = _view_ptrs(views)
    side = _c(side, np.int8)
    H = _c(H, np.float64)
    S = np.zeros((h, w, int(W.sum())), np.uint8)
    offs_c = _c(offs, np.int32) if offs is not None else None
    r = lib().or_ncc_cost_volume(w, h, _p(ref_img), len(arrs), C.cast(ptrs, C.c_void_p), _p(side), cw, ch,
                                 len(G), _p(G), _p(W), _p(H), _p(offs_c), _p(S))
    if r != 0:
        raise ValueError("ncc cost volume: bad arguments (%d)" % r)
    return S


def ncc_cost_pixels(ref_img, views, side, cw, ch, G, W, H, xy, offs=None):
    """NCC cost vectors [n][sum W] of the pixels xy ([n][2] as x, y)."""
    ref_img = _c(ref_img, np.uint8)
    h, w = ref_img.shape
    G = np.asarray(G, np.int32)
    W = np.asarray(W, np.int32)
    xy = _c(xy, np.int32)
    arrs, ptrs = _view_ptrs(views)
    out = np.zeros((len(xy), int(W.sum())), np.uint8)
    r = lib().or_ncc_cost_pixels(w, h, _p(ref_img), len(arrs), C.cast(ptrs, C.c_void_p), _p(_c(side, np.int8)),
                                 cw, ch, len(G), _p(G), _p(W), _p(_c(H, np.float64)),
                                 _p(_c(offs, np.int32) if offs is not None else None), len(xy), _p(xy), _p(out))
    if r != 0:
        raise ValueError("ncc_cost_pixels failed (%d)" % r)
    return out


def ncc_window(a, b):
    """NCC cost of one pair of windows: a uint8 [ch][cw] (reference), b
    float32 [ch][cw] (warped view)."""
    a = _c(a, np.uint8)
    b = _c(b, np.float32)
    ch, cw = a.shape
    return int(lib().or_ncc_window(_p(a), _p(b), cw, ch))


def cost_sample(ct_ref, views, side, cw, ch, G, H, f, g, x, y):
    h, w = ct_ref.shape
    G = np.asarray(G, np.int32)
    arrs, ptrs = _view_ptrs(views)
    return lib().or_cost_sample(w, h, _p(_c(ct_ref, np.uint64)), len(arrs), C.cast(ptrs, C.c_void_p),
                                _p(_c(side, np.int8)), cw, ch, len(G), _p(G), _p(_c(H, np.float64)),
                                int(f), int(g), int(x), int(y))


def cost_pixels(ct_ref, views, side, cw, ch, G, W, H, xy, offs=None):
    """Cost vectors [n][sum W] of the pixels xy ([n][2] as x, y)."""
    h, w = ct_ref.shape
    G = np.asarray(G, np.int32)
    W = np.asarray(W, np.int32)
    xy = _c(xy, np.int32)
    arrs, ptrs = _view_ptrs(views)
    out = np.zeros((len(xy), int(W.sum())), np.uint8)
    r = lib().or_cost_pixels(w, h, _p(_c(ct_ref, np.uint64)), len(arrs), C.cast(ptrs, C.c_void_p),
                             _p(_c(side, np.int8)), cw, ch, len(G), _p(G), _p(W), _p(_c(H, np.float64)),
                             _p(_c(offs, np.int32) if offs is not None else None), len(xy), _p(xy), _p(out))
    if r != 0:
        raise ValueError("cost_pixels failed (%d)" % r)
    return out


def sgm(S, W, p1, lut, ref, n_paths, offs=None, dI=None, want_sbar=True, want_lr=False, pg=None):
    """Semi-global aggregation.  pg: None, or a dict with the level geometry
    (G, fam_delta, fam_n, Kinv, step) to add the path-gradient offsets."""
    h, w, D = S.shape
    W = np.asarray(W, np.int32)
    Sbar = np.zeros((h, w, D), np.uint16) if want_sbar else None
    Lr = np.zeros((n_paths, h, w, D), np.uint16) if want_lr else None
    args = [w, h, len(W), _p(W), _p(_c(offs, np.int32) if offs is not None else None),
            _p(_c(S, np.uint8)), _p(_c(dI, np.int8) if dI is not None else None), int(p1),
            _p(_c(lut, np.int32)), _p(_c(ref, np.uint8)), int(n_paths), _p(Sbar), _p(Lr)]
    if pg is None:
        r = lib().or_sgm(*args)
    else:
        G = np.asarray(pg["G"], np.int32)
        goff = np.concatenate([[0], np.cumsum(G)[:-1]]).astype(np.int32)
        keep = [goff, _c(pg["fam_delta"], np.float64), _c(pg["fam_n"], np.float64), _c(pg["Kinv"], np.float64),
                _c(pg["step"], np.float64)]
        r = lib().or_sgm_pg(*args, 1, *[_p(a) for a in keep])
    if r != 0:
        raise OverflowError("aggregated cost exceeds 16 bits")
    return Sbar, Lr


def wta_refine(Sbar, W, G, fam_n, fam_delta, Kinv, offs=None):
    h, w, D = Sbar.shape
    W = np.asarray(W, np.int32)
    G = np.asarray(G, np.int32)
    label = np.zeros((h, w), np.int32)
    fam = np.zeros((h, w), np.int32)
    depth = np.zeros((h, w), np.float32)
    lib().or_wta_refine(w, h, len(W), _p(W), _p(G), _p(_c(offs, np.int32) if offs is not None else None),
                        _p(_c(Sbar, np.uint16)), _p(_c(fam_n, np.float64)), _p(_c(fam_delta, np.float64)),
                        _p(_c(Kinv, np.float64)), _p(label), _p(fam), _p(depth))
    return label, fam, depth


def median5(d):
    d = _c(d, np.float32)
    out = np.zeros_like(d)
    lib().or_median5(_p(d), d.shape[1], d.shape[0], _p(out))
    return out


def normals(depth, Kinv):
    depth = _c(depth, np.float32)
    h, w = depth.shape
    out = np.zeros((h, w, 3), np.float32)
    lib().or_normals(_p(depth), w, h, _p(_c(Kinv, np.float64)), _p(out))
    return out


def normal_smooth(n, img, radius, beta):
    n = _c(n, np.float32)
    h, w, _ = n.shape
    out = np.zeros_like(n)
    lib().or_normal_smooth(_p(n), _p(_c(img, np.uint8)), w, h, int(radius), float(beta), _p(out))
    return out


def confidence(n, label, fam, fam_n, rho_deg):
    n = _c(n, np.float32)
    h, w, _ = n.shape
    out = np.zeros((h, w), np.float32)
    lib().or_confidence(_p(n), _p(_c(label, np.int32)), _p(_c(fam, np.int32)), _p(_c(fam_n, np.float64)),
                        w, h, float(rho_deg), _p(out))
    return out


def upsample_nn(src, dw, dh):
    src = _c(src, np.float32)
    sh, sw = src.shape[:2]
    ch = 1 if src.ndim == 2 else src.shape[2]
    out = np.zeros((dh, dw) + (() if src.ndim == 2 else (ch,)), np.float32)
    lib().or_upsample_nn(_p(src), sw, sh, ch, dw, dh, _p(out))
    return out


def window_offsets(dbar, Kinv, fam_n, deltas, W):
    """Per-pixel sampling windows; deltas: the level's plane list of every
    family (a list of arrays)."""
    dbar = _c(dbar, np.float32)
    h, w = dbar.shape
    nf = len(deltas)
    G = np.array([len(d) for d in deltas], np.int32)
    cat = _c(np.concatenate([np.asarray(d, np.float64) for d in deltas]), np.float64)
    offs = np.zeros((nf, h, w), np.int32)
    lib().or_window_offsets(_p(dbar), w, h, _p(_c(Kinv, np.float64)), nf, _p(_c(fam_n, np.float64)), _p(cat),
                            _p(G), _p(np.asarray(W, np.int32)), _p(offs))
    return offs


def delta_i(dbar, nbar, Kinv, fam_n, deltas):
    """Surface-normal index offsets; deltas: the level's plane list of every
    family."""
    dbar = _c(dbar, np.float32)
    h, w = dbar.shape
    nf = len(deltas)
    G = np.array([len(d) for d in deltas], np.int32)
    cat = _c(np.concatenate([np.asarray(d, np.float64) for d in deltas]), np.float64)
    out = np.zeros((8, h, w, nf), np.int8)
    lib().or_delta_i(_p(dbar), _p(_c(nbar, np.float32)), w, h, _p(_c(Kinv, np.float64)), nf,
                     _p(_c(fam_n, np.float64)), _p(cat), _p(G), _p(out))
    return out


# ---------------------------------------------------------------------------
# frame driver
# ---------------------------------------------------------------------------

MAX_TOP_PLANES = 256


def family_range(wl, fam):
    """(delta_min, delta_max) of a family: given, or -- when both are 0 --
    the bounding planes of the depth range [depth_min, depth_max] over the
    reference frustum (level-0 intrinsics and size)."""
    lo, hi = float(fam.get("delta_min", 0.0)), float(fam.get("delta_max", 0.0))
    if lo == 0.0 and hi == 0.0:
        return bounding_planes(np.asarray(wl["K"], np.float64), wl["width"], wl["height"], fam["n"],
                               fam["depth_min"], fam["depth_max"])
    return lo, hi


def top_list(wl, fam):
    """The coarsest level's plane list of a family, increasing distances:
    the caller's explicit list ("delta", either order); count > 0: count
    planes uniform in inverse distance over the family's range; count 0:
    the cross-ratio list (Alg. 2, coarsest-level intrinsics and size) of
    the view with the longest one, resampled to 256 planes when longer."""
    if fam.get("delta") is not None:
        d = np.asarray(fam["delta"], np.float64)
        return d[::-1].copy() if d[0] > d[-1] else d.copy()
    lo, hi = family_range(wl, fam)
    if int(fam["count"]) != 0:
        return plane_list(lo, hi, int(fam["count"]))
    n = wl["params"]["n_levels"]
    _, Kt = kinv_level(np.asarray(wl["K"], np.float64), n - 1)
    wt, ht = wl["width"] >> (n - 1), wl["height"] >> (n - 1)
    best = None
    for v in wl["views"]:
        R, t = relative_pose(wl["ref"]["R"], wl["ref"]["t"], v["R"], v["t"])
        try:
            lst = cross_ratio_planes(Kt, wt, ht, R, t, fam["n"], lo, hi)
        except ValueError:
            continue
        if best is None or len(lst) > len(best):
            best = lst
    if best is None or len(best) < 2:
        raise ValueError("no cross-ratio plane list for a family with count 0")
    best = best[::-1].copy()
    if len(best) > MAX_TOP_PLANES:
        best = level_list(best, MAX_TOP_PLANES)
    return best


def family_count(wl, fam):
    """Planes of a family at the coarsest level."""
    return len(top_list(wl, fam))


def level_plan(wl, level):
    """Per-level plane families: plane count, window size, lists, normals.
    Level l has count * 2^(n-1-l) planes interpolated from the coarsest
    list.  ``step`` is the inverse-distance step of lists uniform in inverse
    distance (SGM^Pi-pg), None for other lists."""
    p = wl["params"]
    n = p["n_levels"]
    fams = wl["families"]
    tops = [top_list(wl, f) for f in fams]
    G = [len(t) << (n - 1 - level) for t in tops]
    if level == n - 1 or p["window_labels"] <= 0:
        W = list(G)
    else:
        W = [min(int(p["window_labels"]), g) for g in G]
    deltas = [t.copy() if g == len(t) else level_list(t, g) for t, g in zip(tops, G)]
    fam_n = np.array([f["n"] for f in fams], np.float64)
    uniform = all(f.get("delta") is None and int(f["count"]) != 0 for f in fams)
    step = None
    if uniform:
        step = np.array([(1.0 / d[0] - 1.0 / d[-1]) / (len(d) - 1) for d in deltas])
    return dict(G=G, W=W, deltas=deltas, fam_n=fam_n, step=step)


def subset_multiplier(side):
    nL = sum(1 for s in side if s < 0)
    nR = sum(1 for s in side if s > 0)
    return max(nL, nR)


def run_frame(wl, keep=False, levels_only=None):
    """Run the whole pipeline on a scenegen workload.  Returns the level-0
    depth/normal/confidence plus, with keep=True, every intermediate per
    level.  ``levels_only`` stops after the given level (for bounded runs)."""
    p = wl["params"]
    n = p["n_levels"]
    K = np.asarray(wl["K"], np.float64)
    ref = wl["ref"]
    views = wl["views"]
    side = np.asarray(wl["side"], np.int8)
    ncc = p.get("cost", "census") == "ncc"
    # the NCC cost is a subset mean on the 0..255 scale of one view, the
    # census cost a sum scaled by m: P1 and fixed P2 scale alike
    m = 1 if ncc else subset_multiplier(wl["side"])
    p1 = m * p["p1"]
    lut = p2_lut(p1, p["p2_mode"], m * p["p2_fixed"], p["p2_alpha"], p["p2_beta"])
    cw, chh = p["census_w"], p["census_h"]
    pyr_ref = [np.asarray(ref["img"], np.uint8)]
    pyr_views = [[np.asarray(v["img"], np.uint8)] for v in views]
    for l in range(1, n):
        pyr_ref.append(pyr_down(pyr_ref[-1]))
        for pv in pyr_views:
            pv.append(pyr_down(pv[-1]))
    rel = [relative_pose(ref["R"], ref["t"], v["R"], v["t"]) for v in views]
    out = {"levels": {}}
    offs = None
    dI = None
    for l in range(n - 1, -1, -1):
        Ki, Kl = kinv_level(K, l)
        plan = level_plan(wl, l)
        img = pyr_ref[l]
        h, w = img.shape
        sumG = sum(plan["G"])
        H = np.zeros((len(views), sumG, 3, 3))
        for k, (R, t) in enumerate(rel):
            g0 = 0
            for f, dl in enumerate(plan["deltas"]):
                for j, dv in enumerate(dl):
                    H[k, g0 + j] = homography(Kl, Ki, R, t, plan["fam_n"][f], dv)
                g0 += len(dl)
        ct = None if ncc else census(img, cw, chh)
        top = l == n - 1
        o = None if top or p["window_labels"] <= 0 else offs
        if ncc:
            S = ncc_cost_volume(img, [pv[l] for pv in pyr_views], side, cw, chh, plan["G"], plan["W"], H, o)
        else:
            S = cost_volume(ct, [pv[l] for pv in pyr_views], side, cw, chh, plan["G"], plan["W"], H, o)
        use_dI = (not top) and p["sgm_variant"] == 1 and dI is not None
        fam_delta = np.concatenate(plan["deltas"])
        pg = None
        if p["sgm_variant"] == 2:
            if plan["step"] is None:
                raise ValueError("SGM^Pi-pg needs plane lists uniform in inverse distance")
            pg = dict(G=plan["G"], fam_delta=fam_delta, fam_n=plan["fam_n"], Kinv=Ki, step=plan["step"])
        Sbar, _ = sgm(S, plan["W"], p1, lut, img, p["n_paths"], offs=o, dI=dI if use_dI else None, pg=pg)
        label, fam, depth_raw = wta_refine(Sbar, plan["W"], plan["G"], plan["fam_n"], fam_delta, Ki, o)
        depth = median5(depth_raw) if p["median"] else depth_raw
        nraw = normals(depth, Ki)
        nsm = normal_smooth(nraw, img, p["normal_radius"], p["normal_beta"])
        conf = confidence(nsm, label, fam, plan["fam_n"], p["conf_rho_deg"])
        rec = dict(depth=depth, normal=nsm, conf=conf, label=label, fam=fam)
        if keep:
            rec.update(S=S, Sbar=Sbar, depth_raw=depth_raw, normal_raw=nraw, ct=ct, offs=o,
                       dI=dI if use_dI else None, H=H, plan=plan, img=img)
        out["levels"][l] = rec
        if l > 0:
            fh, fw = pyr_ref[l - 1].shape
            dbar = upsample_nn(depth, fw, fh)
            nbar = upsample_nn(nsm, fw, fh)
            Ki_f, _ = kinv_level(K, l - 1)
            plan_f = level_plan(wl, l - 1)
            offs = window_offsets(dbar, Ki_f, plan_f["fam_n"], plan_f["deltas"], plan_f["W"])
            dI = delta_i(dbar, nbar, Ki_f, plan_f["fam_n"], plan_f["deltas"]) if p["sgm_variant"] == 1 else None
            if keep:
                out["levels"][l]["seed"] = dict(dbar=dbar, nbar=nbar, offs=offs, dI=dI)
        if levels_only is not None and l == levels_only:
            break
    if 0 in out["levels"]:
        lv = out["levels"][0]
        out["depth"], out["normal"], out["conf"] = lv["depth"], lv["normal"], lv["conf"]
        if p.get("dog_filter"):
            keep = dog_mask(pyr_ref[0]).astype(bool)
            out["depth"] = np.where(keep, out["depth"], 0).astype(np.float32)
            out["normal"] = np.where(keep[..., None], out["normal"], 0).astype(np.float32)
            out["conf"] = np.where(keep, out["conf"], 0).astype(np.float32)
    out["pyr_ref"] = pyr_ref
    out["pyr_views"] = pyr_views
    return out


# ----------------------------------------------------------------- post filters
DOG_SIGMA, DOG_RADIUS, DOG_THRESH, DOG_MIN_ON, DOG_MIN_OFF = 1.4, 3, 0.5, 7, 21


def gauss_taps(sigma=DOG_SIGMA, radius=DOG_RADIUS):
    t = np.zeros(2 * radius + 1)
    lib().or_gauss_taps(float(sigma), int(radius), _p(t))
    return t


def dog(img, sigma=DOG_SIGMA, radius=DOG_RADIUS):
    img = _c(img, np.uint8)
    h, w = img.shape
    out = np.zeros((h, w))
    lib().or_dog(_p(img), w, h, float(sigma), int(radius), _p(out))
    return out


def dog_mask(img, sigma=DOG_SIGMA, radius=DOG_RADIUS, thresh=DOG_THRESH, min_on=DOG_MIN_ON, min_off=DOG_MIN_OFF):
    """Texture mask of the DoG filter: 1 textured (keep), 0 weak texture."""
    img = _c(img, np.uint8)
    h, w = img.shape
    m = np.zeros((h, w), np.uint8)
    lib().or_dog_mask(_p(img), w, h, float(sigma), int(radius), float(thresh), int(min_on), int(min_off), _p(m))
    return m


def speckle(mask, value, min_size):
    m = _c(mask, np.uint8).copy()
    h, w = m.shape
    lib().or_speckle(_p(m), w, h, int(value), int(min_size))
    return m


def geo_consistency(K, depth_ref, depth_nb, R, t, eta_r=10.0, eta_h=3):
    """Hits and keep mask of the geometric consistency filter; R, t:
    reference-to-neighbour relative poses [n][3][3], [n][3]."""
    dref = _c(depth_ref, np.float32)
    h, w = dref.shape
    arrs = [_c(d, np.float32) for d in depth_nb]
    ptrs = (C.c_void_p * max(len(arrs), 1))(*[a.ctypes.data for a in arrs])
    hits = np.zeros((h, w), np.int32)
    keep = np.zeros((h, w), np.uint8)
    lib().or_geo_consistency(w, h, _p(_c(K, np.float64)), _p(dref), len(arrs), C.cast(ptrs, C.c_void_p),
                             _p(_c(R, np.float64)), _p(_c(t, np.float64)), float(eta_r), int(eta_h), _p(hits),
                             _p(keep))
    return hits, keep


# ----------------------------------------------------------------- plane set
def bounding_planes(K, w, h, n, d_min, d_max):
    out = np.zeros(2)
    r = lib().or_bounding_planes(_p(_c(K, np.float64)), int(w), int(h), _p(_c(n, np.float64)), float(d_min),
                                 float(d_max), _p(out))
    if r != 0:
        raise ValueError("bounding_planes: bad input")
    return float(out[0]), float(out[1])


def cross_ratio_planes(K, w, h, R, t, n, d_min, d_max, max_planes=4096):
    """Plane distances from delta_max to delta_min with one-pixel image steps
    (Alg. 2); R, t: reference -> view k."""
    out = np.zeros(max_planes)
    cnt = C.c_int(0)
    r = lib().or_cross_ratio_planes(_p(_c(K, np.float64)), int(w), int(h), _p(_c(R, np.float64)),
                                    _p(_c(t, np.float64)), _p(_c(n, np.float64)), float(d_min), float(d_max),
                                    int(max_planes), _p(out), C.byref(cnt))
    if r == -2:
        raise OverflowError(f"cross-ratio list needs {cnt.value} planes")
    if r != 0:
        raise ValueError("cross_ratio_planes: bad input")
    return out[:cnt.value].copy()
