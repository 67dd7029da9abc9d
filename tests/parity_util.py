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


# The sweep's reciprocal of the homogeneous coordinate is the hardware
# estimate refined by two Newton steps: within an ulp of the correctly
# rounded quotient the oracle takes.  A warped sample can then differ from
# the oracle's in the last float bit (rarely: about one sample in a million),
# and a census bit or an NCC rounding only flips at a near tie with it, so
# costs the kernel computes from images agree with the oracle's on all but a
# vanishing fraction of entries.  Costs from the oracle's own warped images
# stay bit-exact.
FROM_IMAGES_MIN_SAME = 0.9999


def assert_costs_from_images(got, exp, what=""):
    """Cost entries computed from images (the kernel warps): identical on
    >= FROM_IMAGES_MIN_SAME of the entries; prints the differing count."""
    same = got == exp
    n_diff = int(same.size - np.count_nonzero(same))
    if n_diff:
        print(f"[costs from images] {what}: {n_diff} of {same.size} entries differ; first {first_mismatch(got, exp)}",
              flush=True)
    assert same.mean() >= FROM_IMAGES_MIN_SAME, (what, n_diff, first_mismatch(got, exp))


# Warped intensities: within 1e-4 on [0, 1] of the oracle's, and identical on
# all but a vanishing fraction of samples (see above).
WARP_TOL = 1e-4 * 255.0


def assert_warp_close(got, exp, what=""):
    d = np.abs(got.astype(np.float64) - exp.astype(np.float64))
    assert d.max() <= WARP_TOL, (what, float(d.max()) / 255.0)
    assert np.mean(got == exp) >= 0.999, (what, float(np.mean(got == exp)))
