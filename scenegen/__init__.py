"""Seeded synthetic scene generator for plane-sweep MVS workloads.

This module only produces *inputs*: rendered grayscale frames, camera poses,
intrinsics, plane families and parameter sets, plus ground truth (depth,
normal, surface id).  It holds none of the matching or optimisation
arithmetic of the method; both the CPU oracle and the GPU library consume
what it renders.

Scene model (stands in for the oblique UAV footage, DTU and 3DOMcity data,
which are not available): a textured ground plane z=0, axis-aligned boxes
and gable-roofed boxes, rendered by ray casting through a pinhole camera.
Texture is uniform noise smoothed with a Gaussian (sigma 1.5 texels),
contrast-stretched to mean 128 / std 40, laid out in world space so that one
texel is about one reference pixel at the median scene depth.

Camera convention: x_cam = R x_world + t; camera axes x right, y down,
z forward; pixel (u, v) has its centre at (u+0.5, v+0.5) in the coordinates
K maps to.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Box", "Scene", "pose_from_heading", "render", "noise_texture",
    "make_workload", "WORKLOADS",
]


# --------------------------------------------------------------------------
# geometry helpers
# --------------------------------------------------------------------------

def _rot_axis(axis, ang):
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    x, y, z = axis
    c, s = math.cos(ang), math.sin(ang)
    C = 1.0 - c
    return np.array([
        [c + x * x * C, x * y * C - z * s, x * z * C + y * s],
        [y * x * C + z * s, c + y * y * C, y * z * C - x * s],
        [z * x * C - y * s, z * y * C + x * s, c + z * z * C],
    ])


def pose_from_heading(C, heading_deg, pitch_deg, roll_deg=0.0):
    """Camera at world position C looking along compass heading (0 = +y,
    90 = +x) pitched down by pitch_deg.  Returns (R, t) with
    x_cam = R x_world + t."""
    C = np.asarray(C, np.float64)
    psi = math.radians(heading_deg)
    th = math.radians(pitch_deg)
    f = np.array([math.sin(psi) * math.cos(th), math.cos(psi) * math.cos(th), -math.sin(th)])
    xr = np.array([math.cos(psi), -math.sin(psi), 0.0])
    if abs(pitch_deg) >= 89.999:          # nadir: keep x along the heading's right
        f = np.array([0.0, 0.0, -1.0]) if pitch_deg > 0 else np.array([0.0, 0.0, 1.0])
    yd = np.cross(f, xr)
    R = np.stack([xr, yd, f])
    if roll_deg:
        R = _rot_axis(f, math.radians(roll_deg)) @ R.T
        R = R.T
    t = -R @ C
    return R, t


@dataclass
class Box:
    x0: float
    x1: float
    y0: float
    y1: float
    h: float                   # wall height (flat roof at z=h)
    roof_h: float = 0.0        # >0: gable roof ridge above h
    ridge_x: bool = True       # ridge runs along x (else along y)


@dataclass
class Scene:
    boxes: list = field(default_factory=list)
    ground_z: float = 0.0


# --------------------------------------------------------------------------
# texture
# --------------------------------------------------------------------------

def noise_texture(seed: int, size: int = 1024, sigma: float = 1.5,
                  mean: float = 128.0, std: float = 40.0) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    t = rng.random((size, size))
    t = gaussian_filter(t, sigma, mode="wrap")
    t = (t - t.mean()) / t.std() * std + mean
    return np.clip(t, 0.0, 255.0)


def _sample_tex(tex, u, v):
    n = tex.shape[0]
    x0 = np.floor(u)
    y0 = np.floor(v)
    fx = u - x0
    fy = v - y0
    x0 = x0.astype(np.int64) % n
    y0 = y0.astype(np.int64) % n
    x1 = (x0 + 1) % n
    y1 = (y0 + 1) % n
    return ((1 - fx) * (1 - fy) * tex[y0, x0] + fx * (1 - fy) * tex[y0, x1]
            + (1 - fx) * fy * tex[y1, x0] + fx * fy * tex[y1, x1])


# --------------------------------------------------------------------------
# ray casting
# --------------------------------------------------------------------------

def _project_rect(K, R, t, pts, w, h):
    """Pixel rectangle covering the projection of 3-D points; None if any
    point is behind the camera (then the whole image is used)."""
    Xc = pts @ R.T + t
    if np.any(Xc[:, 2] <= 1e-6):
        return 0, w, 0, h
    uv = Xc @ K.T
    u = uv[:, 0] / uv[:, 2]
    v = uv[:, 1] / uv[:, 2]
    u0 = max(int(math.floor(u.min())) - 2, 0)
    u1 = min(int(math.ceil(u.max())) + 2, w)
    v0 = max(int(math.floor(v.min())) - 2, 0)
    v1 = min(int(math.ceil(v.max())) + 2, h)
    if u0 >= u1 or v0 >= v1:
        return None
    return u0, u1, v0, v1


def render(scene: Scene, K, R, t, w, h, tex, texel, seed_offsets=0):
    """Ray-cast the scene.  Returns dict with 'img' (float, 0..255),
    'depth' (camera z, inf where nothing is hit), 'normal' (camera coords),
    'surf' (surface id, -1 none)."""
    K = np.asarray(K, np.float64)
    R = np.asarray(R, np.float64)
    t = np.asarray(t, np.float64)
    C = -R.T @ t
    Kinv = np.linalg.inv(K)
    uu, vv = np.meshgrid(np.arange(w) + 0.5, np.arange(h) + 0.5)
    pix = np.stack([uu, vv, np.ones_like(uu)], -1)
    dcam = pix @ Kinv.T                      # camera-frame ray with z = 1
    dw = dcam @ R                             # world ray (R^T d), hit param = depth
    depth = np.full((h, w), np.inf)
    nrm = np.zeros((h, w, 3))
    surf = np.full((h, w), -1, np.int64)
    su = np.zeros((h, w))
    sv = np.zeros((h, w))

    def commit(sl, tt, hitmask, n_world, sid, s_u, s_v):
        r0, r1, c0, c1 = sl
        dsub = depth[r0:r1, c0:c1]
        m = hitmask & (tt > 1e-6) & (tt < dsub)
        if not np.any(m):
            return
        dsub[m] = tt[m]
        nsub = nrm[r0:r1, c0:c1]
        nw = np.broadcast_to(np.asarray(n_world, np.float64), nsub.shape) if np.ndim(n_world) == 1 else n_world
        nsub[m] = (nw @ R.T)[m]
        surf[r0:r1, c0:c1][m] = sid
        su[r0:r1, c0:c1][m] = s_u[m]
        sv[r0:r1, c0:c1][m] = s_v[m]

    # ground plane z = ground_z
    dz = dw[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = (scene.ground_z - C[2]) / dz
    X = C + tg[..., None] * dw
    commit((0, h, 0, w), tg, np.isfinite(tg), np.array([0.0, 0.0, 1.0]), 0, X[..., 0], X[..., 1])

    sid = 1
    for b in scene.boxes:
        top = b.h + b.roof_h
        corners = np.array([[x, y, z] for x in (b.x0, b.x1) for y in (b.y0, b.y1) for z in (0.0, top)])
        rect = _project_rect(K, R, t, corners, w, h)
        if rect is None:
            sid += 8
            continue
        u0, u1, v0, v1 = rect
        sl = (v0, v1, u0, u1)
        d = dw[v0:v1, u0:u1]
        with np.errstate(divide="ignore", invalid="ignore"):
            # walls + flat top of the box body (z in [0, h])
            lo = np.array([b.x0, b.y0, 0.0])
            hi = np.array([b.x1, b.y1, b.h])
            t1 = (lo - C) / d
            t2 = (hi - C) / d
            tmin = np.minimum(t1, t2)
            tmax = np.maximum(t1, t2)
            tnear = np.nanmax(tmin, axis=-1)
            tfar = np.nanmin(tmax, axis=-1)
            hit = (tnear <= tfar) & (tfar > 0)
            ax = np.nanargmax(tmin, axis=-1)
            Xh = C + tnear[..., None] * d
            for a in range(3):
                for sgn in (-1.0, 1.0):
                    if a == 2 and sgn < 0:
                        continue
                    if a == 2 and b.roof_h > 0:
                        continue              # top hidden under the gable roof
                    nw = np.zeros(3)
                    nw[a] = sgn
                    facing = (d[..., a] * sgn) < 0
                    m = hit & (ax == a) & facing
                    if a == 0:
                        s_u, s_v = Xh[..., 1], Xh[..., 2]
                    elif a == 1:
                        s_u, s_v = Xh[..., 0], Xh[..., 2]
                    else:
                        s_u, s_v = Xh[..., 0], Xh[..., 1]
                    commit(sl, tnear, m, nw, sid, s_u, s_v)
                    sid += 1
            if b.roof_h > 0:
                # two roof planes through the ridge, plus the two gable ends
                if b.ridge_x:
                    ym = 0.5 * (b.y0 + b.y1)
                    half = 0.5 * (b.y1 - b.y0)
                    s = b.roof_h / half
                    for side in (-1.0, 1.0):
                        # z = h + roof_h - s*side*(y - ym) on side of ridge
                        nw = np.array([0.0, s * side, 1.0])
                        nw /= np.linalg.norm(nw)
                        # plane: s*side*(y-ym) + (z - h - roof_h) = 0
                        num = -(s * side * (C[1] - ym) + (C[2] - b.h - b.roof_h))
                        den = s * side * d[..., 1] + d[..., 2]
                        tr = num / den
                        Xr = C + tr[..., None] * d
                        m = ((Xr[..., 0] >= b.x0) & (Xr[..., 0] <= b.x1)
                             & ((Xr[..., 1] - ym) * side >= 0) & ((Xr[..., 1] - ym) * side <= half))
                        m &= (nw @ d.reshape(-1, 3).T).reshape(m.shape) < 0
                        commit(sl, tr, m, nw, sid, Xr[..., 0],
                               np.abs(Xr[..., 1] - ym) * math.sqrt(1 + s * s))
                        sid += 1
                    for xe, sgn in ((b.x0, -1.0), (b.x1, 1.0)):
                        te = (xe - C[0]) / d[..., 0]
                        Xe = C + te[..., None] * d
                        zroof = b.h + b.roof_h - s * np.abs(Xe[..., 1] - ym)
                        m = ((Xe[..., 1] >= b.y0) & (Xe[..., 1] <= b.y1)
                             & (Xe[..., 2] >= b.h) & (Xe[..., 2] <= zroof) & (d[..., 0] * sgn < 0))
                        commit(sl, te, m, np.array([sgn, 0.0, 0.0]), sid, Xe[..., 1], Xe[..., 2])
                        sid += 1
                else:
                    xm = 0.5 * (b.x0 + b.x1)
                    half = 0.5 * (b.x1 - b.x0)
                    s = b.roof_h / half
                    for side in (-1.0, 1.0):
                        nw = np.array([s * side, 0.0, 1.0])
                        nw /= np.linalg.norm(nw)
                        num = -(s * side * (C[0] - xm) + (C[2] - b.h - b.roof_h))
                        den = s * side * d[..., 0] + d[..., 2]
                        tr = num / den
                        Xr = C + tr[..., None] * d
                        m = ((Xr[..., 1] >= b.y0) & (Xr[..., 1] <= b.y1)
                             & ((Xr[..., 0] - xm) * side >= 0) & ((Xr[..., 0] - xm) * side <= half))
                        m &= (nw @ d.reshape(-1, 3).T).reshape(m.shape) < 0
                        commit(sl, tr, m, nw, sid, Xr[..., 1],
                               np.abs(Xr[..., 0] - xm) * math.sqrt(1 + s * s))
                        sid += 1
                    for ye, sgn in ((b.y0, -1.0), (b.y1, 1.0)):
                        te = (ye - C[1]) / d[..., 1]
                        Xe = C + te[..., None] * d
                        zroof = b.h + b.roof_h - s * np.abs(Xe[..., 0] - xm)
                        m = ((Xe[..., 0] >= b.x0) & (Xe[..., 0] <= b.x1)
                             & (Xe[..., 2] >= b.h) & (Xe[..., 2] <= zroof) & (d[..., 1] * sgn < 0))
                        commit(sl, te, m, np.array([0.0, sgn, 0.0]), sid, Xe[..., 0], Xe[..., 2])
                        sid += 1
        sid = max(sid, 1)

    # texture lookup: per-surface offset so that surfaces do not repeat
    rng = np.random.default_rng(12345 + seed_offsets)
    offs = rng.uniform(0, tex.shape[0], size=(int(surf.max()) + 2, 2))
    valid = surf >= 0
    img = np.zeros((h, w))
    ids = np.where(valid, surf, 0)
    img[valid] = _sample_tex(tex, su[valid] / texel + offs[ids[valid], 0],
                             sv[valid] / texel + offs[ids[valid], 1])
    return {"img": img, "depth": depth, "normal": nrm, "surf": surf}


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def _K(fx, fy, cx, cy):
    return np.array([[fx, 0.0, cx], [0.0, fy, cy], [0.0, 0.0, 1.0]])


def _place_boxes(rng, n, region, size_rng, height_rng, n_roofs=0, roof_rng=(0.2, 0.5)):
    """Non-overlapping axis-aligned boxes inside region=(x0,x1,y0,y1)."""
    boxes = []
    tries = 0
    while len(boxes) < n and tries < 20000:
        tries += 1
        sx = rng.uniform(*size_rng)
        sy = rng.uniform(*size_rng)
        x0 = rng.uniform(region[0], region[1] - sx)
        y0 = rng.uniform(region[2], region[3] - sy)
        cand = (x0 - 1.0, x0 + sx + 1.0, y0 - 1.0, y0 + sy + 1.0)
        if any(not (cand[1] < b.x0 or cand[0] > b.x1 or cand[3] < b.y0 or cand[2] > b.y1) for b in boxes):
            continue
        boxes.append(Box(x0, x0 + sx, y0, y0 + sy, float(rng.uniform(*height_rng))))
    for i in range(min(n_roofs, len(boxes))):
        b = boxes[i]
        b.ridge_x = bool(rng.integers(0, 2))
        span = (b.y1 - b.y0) if b.ridge_x else (b.x1 - b.x0)
        slope = math.radians(rng.uniform(20.0, 40.0))
        b.roof_h = 0.5 * span * math.tan(slope)
    return boxes


def _frame(scene, K, R, t, w, h, tex, texel, noise_std, rng):
    r = render(scene, K, R, t, w, h, tex, texel)
    img = r["img"]
    if noise_std > 0:
        img = img + rng.normal(0.0, noise_std, img.shape)
    img = np.clip(np.floor(img + 0.5), 0, 255).astype(np.uint8)
    return img, r


def _params(**kw):
    p = dict(n_levels=1, census_w=5, census_h=5, n_paths=8, sgm_variant=0,
             p1=8, p2_mode=0, p2_fixed=64, p2_alpha=8.0, p2_beta=10.0,
             window_labels=0, median=1, normal_radius=2, normal_beta=10.0,
             conf_rho_deg=60.0)
    p.update(kw)
    return p


def _pack(name, K, w, h, imgs, poses, ref_index, side, families, params, gt, scene=None):
    ref_img = imgs[ref_index]
    views = [dict(img=imgs[i], R=poses[i][0], t=poses[i][1]) for i in range(len(imgs)) if i != ref_index]
    return dict(name=name, K=K, width=w, height=h,
                ref=dict(img=ref_img, R=poses[ref_index][0], t=poses[ref_index][1]),
                views=views, side=list(side), families=families, params=params, gt=gt,
                scene=scene)


def config1(seed: int = 0, w: int = 160, h: int = 120):
    """160x120 reference + 2 matching frames translated +-2 m along world x,
    45 deg oblique at 50 m, ground + 4 boxes; 32 fronto-parallel planes
    uniform in inverse depth over [30, 120] m; census 5x5; P1=8, P2=64."""
    rng = np.random.default_rng(seed)
    s = w / 160.0
    K = _K(150.0 * s, 150.0 * s, 80.0 * s, 60.0 * s)
    C = np.array([0.0, 0.0, 50.0])
    R, t = pose_from_heading(C, 0.0, 45.0)
    # ground footprint of this camera is roughly y in [21, 117], |x| < 0.5*y
    boxes = _place_boxes(rng, 4, (-25.0, 25.0, 35.0, 85.0), (8.0, 15.0), (5.0, 20.0))
    scene = Scene(boxes)
    texel = 70.0 / K[0, 0]
    tex = noise_texture(seed + 1000)
    poses, imgs = [], []
    for dx in (-2.0, 0.0, 2.0):
        Rk, tk = pose_from_heading(C + np.array([dx, 0.0, 0.0]), 0.0, 45.0)
        img, r = _frame(scene, K, Rk, tk, w, h, tex, texel, 0.0, rng)
        poses.append((Rk, tk))
        imgs.append(img)
        if dx == 0.0:
            gt = dict(depth=r["depth"], normal=r["normal"], surf=r["surf"])
    fam = [dict(n=(0.0, 0.0, -1.0), delta_min=30.0, delta_max=120.0, count=32)]
    params = _params(n_levels=1, census_w=5, census_h=5, p1=8, p2_mode=0, p2_fixed=64)
    return _pack("config1", K, w, h, imgs, poses, 1, (-1, 1), fam, params, gt, scene)


def _flight(rng, C_ref, heading, n_frames, ref_index, spacing_rng, along_x=True):
    """Smooth flight path: positions spaced U(spacing) metres along a gently
    curving, slightly climbing track through C_ref.  Compass angles are
    measured from +y toward +x; the track runs roughly along the camera's
    x axis (sideways-looking oblique camera)."""
    a0 = math.radians(heading + (90.0 if along_x else 0.0) + rng.uniform(-15.0, 15.0))
    kappa = rng.uniform(-0.01, 0.01)           # rad per metre
    climb = rng.uniform(-0.03, 0.03)
    gaps = rng.uniform(*spacing_rng, size=n_frames - 1)
    arc = np.concatenate([[0.0], np.cumsum(gaps)])
    arc = arc - arc[ref_index]
    centers = []
    for s in arc:
        a = a0 + kappa * s
        if abs(kappa) > 1e-9:
            dx = (math.cos(a0) - math.cos(a)) / kappa
            dy = (math.sin(a) - math.sin(a0)) / kappa
        else:
            dx, dy = s * math.sin(a0), s * math.cos(a0)
        centers.append(C_ref + np.array([dx, dy, climb * s]))
    return centers


def oblique_urban(seed: int, w: int, h: int, fx: float, n_views: int, n_boxes: int,
                  n_roofs: int, height: float = 60.0, pitch: float = 45.0,
                  noise_frac: float = 0.05, spacing=(1.0, 4.0)):
    rng = np.random.default_rng(seed)
    K = _K(fx, fx, w / 2.0, h / 2.0)
    heading = float(rng.uniform(0.0, 360.0))
    C_ref = np.array([0.0, 0.0, height])
    R0, t0 = pose_from_heading(C_ref, heading, pitch)
    # ground footprint: intersect the four corner rays with z=0
    Kinv = np.linalg.inv(K)
    pts = []
    for (u, v) in ((0, 0), (w, 0), (0, h), (w, h), (w / 2, h / 2)):
        d = R0.T @ (Kinv @ np.array([u, v, 1.0]))
        tt = -height / d[2]
        pts.append(C_ref + tt * d)
    pts = np.array(pts)
    # boxes in the local frame of the footprint (axis aligned in world)
    region = (pts[:, 0].min() * 0.8, pts[:, 0].max() * 0.8, pts[:, 1].min() * 0.8, pts[:, 1].max() * 0.8)
    # axis-aligned region is generous; shrink toward the central footprint
    cx = pts[4, 0]
    cy = pts[4, 1]
    half = 0.35 * min(region[1] - region[0], region[3] - region[2])
    region = (cx - half, cx + half, cy - half, cy + half)
    boxes = _place_boxes(rng, n_boxes, region, (8.0, 25.0), (5.0, 30.0), n_roofs)
    scene = Scene(boxes)
    texel = float(np.median(np.linalg.norm(pts[:4] - C_ref, axis=1))) * 0.75 / fx
    tex = noise_texture(seed + 1000, size=2048)
    n_frames = n_views + 1
    ref_index = n_frames // 2
    centers = _flight(rng, C_ref, heading, n_frames, ref_index, spacing)
    imgs, poses, gt = [], [], None
    for i, C in enumerate(centers):
        if i == ref_index:
            R, t = R0, t0
        else:
            R, t = pose_from_heading(C, heading + rng.uniform(-1.0, 1.0), pitch + rng.uniform(-1.0, 1.0),
                                     rng.uniform(-1.0, 1.0))
        img, r = _frame(scene, K, R, t, w, h, tex, texel, noise_frac * 255.0, rng)
        imgs.append(img)
        poses.append((R, t))
        if i == ref_index:
            gt = dict(depth=r["depth"], normal=r["normal"], surf=r["surf"])
    side = [-1] * ref_index + [1] * (n_frames - 1 - ref_index)
    return K, imgs, poses, ref_index, side, gt, scene, R0


def ground_normal_cam(R):
    """World up-normal (0,0,1) as a plane normal in camera coordinates,
    oriented to face the camera (negative z component)."""
    n = R @ np.array([0.0, 0.0, 1.0])
    if n[2] > 0:
        n = -n
    return n


def config2(seed: int = 1, w: int = 1920, h: int = 1080, planes: int = 128, window: int = 128):
    """1920x1080 reference + 4 views on an oblique urban scene (40 boxes,
    10 gable roofs), 5% noise, 3 levels, 128 fronto-parallel planes per level
    over [20, 400] m, census 9x7, surface-aware 8-path SGM with adaptive P2."""
    s = w / 1920.0
    K, imgs, poses, ref_index, side, gt, scene, _ = oblique_urban(
        seed, w, h, 1500.0 * s, 4, 40, 10)
    fam = [dict(n=(0.0, 0.0, -1.0), delta_min=20.0, delta_max=400.0, count=planes)]
    params = _params(n_levels=3, census_w=9, census_h=7, p1=24, p2_mode=1,
                     sgm_variant=1, window_labels=window)
    return _pack("config2", K, w, h, imgs, poses, ref_index, side, fam, params, gt, scene)


def _tilt(n, axis_cam, deg):
    Rt = _rot_axis(axis_cam, math.radians(deg))
    m = Rt @ n
    return m / np.linalg.norm(m)


def plane_families(R_ref, K, w, h, d_min, d_max, count, n_families=4):
    """Fronto-parallel, the ground normal and the ground normal tilted by
    +-20 deg (about the camera x axis), each with its own distance range
    covering the depth range [d_min, d_max] over the image."""
    ng = ground_normal_cam(R_ref)
    normals = [np.array([0.0, 0.0, -1.0]), ng, _tilt(ng, [1.0, 0.0, 0.0], 20.0),
               _tilt(ng, [1.0, 0.0, 0.0], -20.0)][:n_families]
    Kinv = np.linalg.inv(K)
    fams = []
    for n in normals:
        # distance range: delta = -n^T X over the frustum corners between d_min and d_max
        ds = []
        for (u, v) in ((0, 0), (w, 0), (0, h), (w, h), (w / 2, h / 2)):
            ray = Kinv @ np.array([u, v, 1.0])
            for d in (d_min, d_max):
                ds.append(-(n @ (d * ray)))
        ds = np.array(ds)
        lo = max(float(ds.min()), 0.25 * d_min)
        hi = float(ds.max())
        fams.append(dict(n=tuple(float(x) for x in n), delta_min=lo, delta_max=hi, count=count))
    return fams


def config3(seed: int = 2, w: int = 2704, h: int = 1520, planes: int = 96, window: int = 96,
            n_families: int = 4):
    s = w / 2704.0
    K, imgs, poses, ref_index, side, gt, scene, R0 = oblique_urban(
        seed, w, h, 1500.0 * 1.408 * s, 4, 40, 10)
    fams = plane_families(R0, K, w, h, 20.0, 400.0, planes, n_families)
    params = _params(n_levels=3, census_w=9, census_h=7, p1=24, p2_mode=1,
                     sgm_variant=1, window_labels=window)
    return _pack("config3", K, w, h, imgs, poses, ref_index, side, fams, params, gt, scene)


def nadir_planar(seed: int = 7, w: int = 160, h: int = 120):
    """Noise-free nadir view over flat-roofed boxes on the ground, built so
    that the ground and every roof lie exactly on sweep planes with integer
    disparity (baseline 2 m, fx 200, planes 1/delta = 1/25 - j/800)."""
    rng = np.random.default_rng(seed)
    K = _K(200.0, 200.0, w / 2.0, h / 2.0)
    # plane j has disparity 16 - j/2 px for a 2 m baseline; even j -> integer
    def delta(j):
        return 1.0 / (1.0 / 25.0 - j / 800.0)
    H = delta(16)                      # ground at 50 m
    roofs = [delta(8), delta(12), delta(14), delta(10)]
    boxes = []
    half_w = 0.5 * w / 200.0 * H
    half_h = 0.5 * h / 200.0 * H
    cells = [(-0.55, -0.5), (0.05, -0.5), (-0.55, 0.05), (0.05, 0.05)]
    for (cxf, cyf), dr in zip(cells, roofs):
        sx = rng.uniform(0.25, 0.4) * half_w
        sy = rng.uniform(0.25, 0.4) * half_h
        x0 = cxf * half_w + rng.uniform(0.05, 0.1) * half_w
        y0 = cyf * half_h + rng.uniform(0.05, 0.1) * half_h
        boxes.append(Box(x0, x0 + sx, y0, y0 + sy, H - dr))
    scene = Scene(boxes)
    tex = noise_texture(seed + 1000)
    texel = H / 200.0
    imgs, poses = [], []
    for dx in (-2.0, 0.0, 2.0):
        C = np.array([dx, 0.0, H])
        R, t = pose_from_heading(C, 0.0, 90.0)
        r = render(scene, K, R, t, w, h, tex, texel)
        imgs.append(np.clip(np.floor(r["img"] + 0.5), 0, 255).astype(np.uint8))
        poses.append((R, t))
        if dx == 0.0:
            gt = dict(depth=r["depth"], normal=r["normal"], surf=r["surf"])
    fam = [dict(n=(0.0, 0.0, -1.0), delta_min=25.0, delta_max=100.0, count=25)]
    params = _params(n_levels=1, census_w=5, census_h=5, p1=8, p2_mode=0, p2_fixed=64)
    wl = _pack("nadir_planar", K, w, h, imgs, poses, 1, (-1, 1), fam, params, gt, scene)
    wl["gt_plane_delta"] = [delta(j) for j in range(25)]
    return wl


CONFIG4_SIZES = [(640, 480), (960, 540), (1280, 720), (1920, 1080)]
CONFIG4_SEEDS = list(range(100, 116))


def config4_frame(seed: int):
    """One frame of the uneven batch: resolution drawn from four UAV video
    sizes, 2-5 matching views (split as evenly as possible, the extra one on
    the left), 64-192 planes per level in steps of 8 over [20, 400] m (the
    window at finer levels as wide as the top list), 2 or 3 pyramid levels;
    census 9x7, SGM^Pi-sn, adaptive P2; an independent urban scene per seed."""
    rng = np.random.default_rng(seed)
    w, h = CONFIG4_SIZES[int(rng.integers(len(CONFIG4_SIZES)))]
    n_views = int(rng.integers(2, 6))
    planes = 8 * int(rng.integers(8, 25))
    levels = int(rng.integers(2, 4))
    s = w / 1920.0
    K, imgs, poses, ref_index, side, gt, scene, _ = oblique_urban(seed, w, h, 1500.0 * s, n_views, 40, 10)
    fam = [dict(n=(0.0, 0.0, -1.0), delta_min=20.0, delta_max=400.0, count=planes)]
    params = _params(n_levels=levels, census_w=9, census_h=7, p1=24, p2_mode=1, sgm_variant=1,
                     window_labels=planes)
    return _pack(f"config4_{seed}", K, w, h, imgs, poses, ref_index, side, fam, params, gt, scene)


WORKLOADS = {
    "config1": lambda: config1(0),
    "config2": lambda: config2(1),
    "config3": lambda: config3(2),
    # config-2 shaped cases small enough for the oracle to finish in seconds
    "config2_small": lambda: config2(1, 320, 184, planes=32, window=32),
    "config2_ragged": lambda: config2(5, 333, 187, planes=32, window=16),
    "config3_small": lambda: config3(2, 320, 180, planes=16, window=16),
    "nadir_planar": lambda: nadir_planar(7),
    # the NCC matching cost (5x5 window, phi1 = 100 as in the paper's NCC
    # experiments; fixed P2 of config 1 scaled the same way)
    "config1_ncc": lambda: with_ncc(config1(0), p2_fixed=400),
    "config2_small_ncc": lambda: with_ncc(config2(1, 320, 184, planes=32, window=32)),
    "config2_ncc": lambda: with_ncc(config2(1)),
    "config2_pg": lambda: with_sgm_variant(config2(1), 2),
    # plane counts from the cross-ratio construction (count 0)
    **{f"config4_{sd}": (lambda sd=sd: config4_frame(sd)) for sd in CONFIG4_SEEDS},
    "config1_xr": lambda: with_cross_ratio_counts(config1(0)),
    "config2_small_xr": lambda: with_cross_ratio_counts(config2(1, 320, 184, planes=32, window=32)),
    # an explicit list of varying spacing (geometric distances over the range)
    "config2_small_list": lambda: with_geometric_lists(config2(1, 320, 184, planes=32, window=32)),
    # slanted families given by the depth range only (bounding planes)
    "config3_small_range": lambda: with_depth_range(config3(2, 320, 180, planes=16, window=16), 20.0, 400.0),
}


def served_stream(seed: int, w: int, h: int, n_frames: int, spacing: float = 0.5, planes: int = 128,
                  n_boxes: int = 20, n_roofs: int = 5):
    """One UAV stream of the served workload: n_frames along a smooth
    oblique flight path, spacing metres apart (5 m/s at 10 Hz: 0.5 m), over
    an independent urban scene (seed), fx = 1500 scaled to the width; 3
    levels x planes fronto-parallel planes over [20, 400] m, census 9x7,
    SGM^Pi-sn.  Returns K, frames [(img, R, t)], families, params."""
    s = w / 1920.0
    K, imgs, poses, ref_index, side, gt, scene, _ = oblique_urban(
        seed, w, h, 1500.0 * s, n_frames - 1, n_boxes, n_roofs, spacing=(spacing, spacing))
    fam = [dict(n=(0.0, 0.0, -1.0), delta_min=20.0, delta_max=400.0, count=planes)]
    params = _params(n_levels=3, census_w=9, census_h=7, p1=24, p2_mode=1, sgm_variant=1, window_labels=planes)
    frames = [(img, R, t) for img, (R, t) in zip(imgs, poses)]
    return dict(K=K, width=w, height=h, frames=frames, families=fam, params=params)


SERVED_STREAMS = [(200, 960, 540), (201, 1280, 720), (202, 1920, 1080), (203, 2704, 1520)]


def served_path(seed: int, w: int, h: int, n_frames: int, spacing: float = 0.5, planes: int = 128,
                n_boxes: int = 20, n_roofs: int = 5):
    """A served stream without its images: the scene, intrinsics and the
    poses of n_frames along a smooth oblique flight path (spacing metres
    apart: 5 m/s at 10 Hz), centred on the scene; each image is rendered by
    served_image (independently, so frames can be rendered in parallel)."""
    rng = np.random.default_rng(seed)
    fx = 1500.0 * w / 1920.0
    height, pitch = 60.0, 45.0
    K = _K(fx, fx, w / 2.0, h / 2.0)
    heading = float(rng.uniform(0.0, 360.0))
    C_ref = np.array([0.0, 0.0, height])
    R0, t0 = pose_from_heading(C_ref, heading, pitch)
    Kinv = np.linalg.inv(K)
    pts = []
    for (u, v) in ((0, 0), (w, 0), (0, h), (w, h), (w / 2, h / 2)):
        d = R0.T @ (Kinv @ np.array([u, v, 1.0]))
        pts.append(C_ref + (-height / d[2]) * d)
    pts = np.array(pts)
    region = (pts[:, 0].min() * 0.8, pts[:, 0].max() * 0.8, pts[:, 1].min() * 0.8, pts[:, 1].max() * 0.8)
    cx, cy = pts[4, 0], pts[4, 1]
    half = 0.35 * min(region[1] - region[0], region[3] - region[2])
    boxes = _place_boxes(rng, n_boxes, (cx - half, cx + half, cy - half, cy + half), (8.0, 25.0), (5.0, 30.0),
                         n_roofs)
    texel = float(np.median(np.linalg.norm(pts[:4] - C_ref, axis=1))) * 0.75 / fx
    centers = _flight(rng, C_ref, heading, n_frames, n_frames // 2, (spacing, spacing))
    poses = [pose_from_heading(C, heading + rng.uniform(-1.0, 1.0), pitch + rng.uniform(-1.0, 1.0),
                               rng.uniform(-1.0, 1.0)) for C in centers]
    fam = [dict(n=(0.0, 0.0, -1.0), delta_min=20.0, delta_max=400.0, count=planes)]
    params = _params(n_levels=3, census_w=9, census_h=7, p1=24, p2_mode=1, sgm_variant=1, window_labels=planes)
    return dict(seed=seed, K=K, width=w, height=h, scene=Scene(boxes), texel=texel, poses=poses, families=fam,
                params=params, noise_std=0.05 * 255.0)


_TEX_CACHE = {}


def served_image(path: dict, i: int) -> np.ndarray:
    """Image i of a served stream (its noise drawn from a generator of its
    own, so any subset renders the same)."""
    key = path["seed"]
    if key not in _TEX_CACHE:
        _TEX_CACHE.clear()
        _TEX_CACHE[key] = noise_texture(key + 1000, size=2048)
    R, t = path["poses"][i]
    img, _ = _frame(path["scene"], path["K"], R, t, path["width"], path["height"], _TEX_CACHE[key], path["texel"],
                    path["noise_std"], np.random.default_rng([path["seed"], i]))
    return img


def with_cross_ratio_counts(wl):
    """The same bundle with every family's coarsest plane count left to the
    cross-ratio construction (count 0)."""
    return dict(wl, families=[dict(f, count=0) for f in wl["families"]])


def with_geometric_lists(wl):
    """The same bundle with every family's coarsest list given explicitly:
    count distances in geometric progression over [delta_min, delta_max]
    (denser in distance near the camera, sparser in inverse distance there
    than a list uniform in inverse distance)."""
    fams = []
    for f in wl["families"]:
        n = int(f["count"])
        d = f["delta_min"] * (f["delta_max"] / f["delta_min"]) ** (np.arange(n) / (n - 1))
        fams.append(dict(n=f["n"], delta=[float(x) for x in d], count=n))
    return dict(wl, families=fams)


def with_depth_range(wl, depth_min: float, depth_max: float):
    """The same bundle with every family's distance range left to the
    bounding planes of the depth range (delta_min = delta_max = 0)."""
    fams = [dict(n=f["n"], delta_min=0.0, delta_max=0.0, depth_min=depth_min, depth_max=depth_max,
                 count=f["count"]) for f in wl["families"]]
    return dict(wl, families=fams)


def with_sgm_variant(wl, variant: int):
    """The same bundle with another SGM smoothness term (0 Pi, 1 Pi-sn,
    2 Pi-pg)."""
    return dict(wl, params=dict(wl["params"], sgm_variant=variant))


def with_ncc(wl, window: int = 5, p1: int = 100, p2_fixed: int | None = None):
    """The same bundle matched with the negated, truncated and scaled NCC."""
    params = dict(wl["params"], cost="ncc", census_w=window, census_h=window, p1=p1)
    if p2_fixed is not None:
        params["p2_fixed"] = p2_fixed
    return dict(wl, params=params)


def make_workload(name: str, cache_dir: str | None = None):
    """Render a named workload.  With cache_dir (or FASSMVS_SCENE_CACHE) the
    rendered bundle (images, poses, intrinsics, families, parameters, ground
    truth) is kept in a pickle-free .npz and reused."""
    import json
    import os
    cache_dir = cache_dir or os.environ.get("FASSMVS_SCENE_CACHE")
    if not cache_dir:
        return WORKLOADS[name]()
    path = os.path.join(cache_dir, f"{name}.npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        nv = int(z["n_views"])
        fams = json.loads(str(z["families"]))
        wl = dict(name=name, K=z["K"], width=int(z["width"]), height=int(z["height"]),
                  ref=dict(img=z["ref"], R=z["R_ref"], t=z["t_ref"]),
                  views=[dict(img=z[f"view{i}"], R=z["R_views"][i], t=z["t_views"][i]) for i in range(nv)],
                  side=[int(v) for v in z["side"]], families=fams, params=json.loads(str(z["params"])),
                  gt=dict(depth=z["depth"], normal=z["normal"], surf=z["surf"]), scene=None)
        return wl
    wl = WORKLOADS[name]()
    os.makedirs(cache_dir, exist_ok=True)
    arrs = {"ref": wl["ref"]["img"], "R_ref": np.asarray(wl["ref"]["R"]), "t_ref": np.asarray(wl["ref"]["t"]),
            "R_views": np.array([v["R"] for v in wl["views"]]), "t_views": np.array([v["t"] for v in wl["views"]]),
            "n_views": np.array(len(wl["views"])), "side": np.array(wl["side"]), "K": np.asarray(wl["K"]),
            "width": np.array(wl["width"]), "height": np.array(wl["height"]),
            "families": np.array(json.dumps([dict(f, n=[float(x) for x in f["n"]]) for f in wl["families"]])),
            "params": np.array(json.dumps(wl["params"])),
            "depth": wl["gt"]["depth"], "normal": wl["gt"]["normal"], "surf": wl["gt"]["surf"]}
    for i, v in enumerate(wl["views"]):
        arrs[f"view{i}"] = v["img"]
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrs)
    os.replace(tmp, path)
    return wl
