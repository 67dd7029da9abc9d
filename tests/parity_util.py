"""Comparison helpers shared by the GPU parity tests."""
import numpy as np


def stencil_agree(agree, radius):
    """Pixels whose whole (2 radius + 1)^2 neighbourhood agrees (outside the
    image counts as agreeing): the pixels whose stencil outputs (normals,
    smoothing, confidence) must match when their inputs do."""
    from scipy.ndimage import binary_erosion
    k = 2 * radius + 1
    return binary_erosion(agree, structure=np.ones((k, k), bool), border_value=1)


def compare_level(got, exp, normal_radius=2, min_label=0.999, min_cover=0.99, tol=1e-4):
    """Maps of one level (dicts with label, depth, normal, conf) against the
    oracle's: labels identical on >= min_label of the pixels, depth within
    1e-3 relative where the labels agree, normals and confidence within tol
    on the pixels whose depth stencil agrees (normals use the depth of the
    neighbours, smoothing the normals of a (2r+1)^2 window), which must
    cover >= min_cover of the level.  Returns a small report."""
    agree = got["label"] == exp["label"]
    rep = {"labels": float(agree.mean())}
    assert agree.mean() >= min_label, rep
    ok = agree & (exp["depth"] > 0)
    rel = np.abs(got["depth"][ok] - exp["depth"][ok]) / exp["depth"][ok]
    rep["depth_max_rel"] = float(rel.max()) if rel.size else 0.0
    assert rel.size == 0 or rel.max() <= 1e-3, rep
    dsame = np.abs(got["depth"] - exp["depth"]) <= 1e-6 * np.maximum(exp["depth"], 1e-6)
    st = stencil_agree(dsame & agree, normal_radius + 1)
    rep["stencil_cover"] = float(st.mean())
    assert st.mean() >= min_cover, rep
    dn = np.abs(got["normal"] - exp["normal"]).max(axis=-1)[st]
    dc = np.abs(got["conf"] - exp["conf"])[st]
    rep["normal_max"] = float(dn.max()) if dn.size else 0.0
    rep["conf_max"] = float(dc.max()) if dc.size else 0.0
    assert rep["normal_max"] <= tol and rep["conf_max"] <= tol, rep
    return rep


def first_mismatch(got, exp):
    """Index tuple and values of the first differing entry, or None."""
    d = np.argwhere(got != exp)
    if not len(d):
        return None
    i = tuple(int(v) for v in d[0])
    return i, got[i], exp[i]
