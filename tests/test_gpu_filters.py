"""Parity of the post-processing filters (DoG texture mask, geometric
consistency) with the oracle, through the C ABI."""
import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fm():
    import paper_2112_00821_amd as fm
    return fm


@pytest.fixture(scope="module")
def hd(fm):
    with fm.Handle() as h:
        yield h


def _images():
    rng = np.random.default_rng(4)
    yield "config1", scenegen.make_workload("config1")["ref"]["img"]
    yield "config2_small", scenegen.make_workload("config2_small")["ref"]["img"]
    # flat background with textured patches and specks of every size
    img = np.full((97, 131), 128, np.uint8)
    img[10:40, 10:60] = rng.integers(0, 256, (30, 50))
    img[60:90, 70:120] = (rng.random((30, 50)) * 6 + 125).astype(np.uint8)   # low contrast
    for i in range(40):
        y, x = rng.integers(0, 97), rng.integers(0, 131)
        img[y:y + 1 + i % 3, x:x + 1 + i % 4] = rng.integers(0, 256)
    yield "specks", img


@pytest.mark.parametrize("case", range(3))
def test_dog_mask_and_invalidation_bit_exact(orc, hd, case):
    name, img = list(_images())[case]
    h, w = img.shape
    exp = orc.dog_mask(img)
    rng = np.random.default_rng(case)
    depth = rng.random((h, w)).astype(np.float32) + 1
    normal = rng.random((h, w, 3)).astype(np.float32)
    conf = rng.random((h, w)).astype(np.float32)
    dd, nd, cd = hd.upload(depth), hd.upload(normal), hd.upload(conf)
    mask = hd.filter_dog(hd.upload(img), dd, nd, cd).numpy()
    assert np.array_equal(mask, exp), (name, np.mean(mask != exp))
    keep = exp.astype(bool)
    assert np.array_equal(dd.numpy(), np.where(keep, depth, 0))
    assert np.array_equal(nd.numpy(), np.where(keep[..., None], normal, 0))
    assert np.array_equal(cd.numpy(), np.where(keep, conf, 0))


def _plane_maps(rng, noise):
    w, h = 96, 72
    K = np.array([[90.0, 0, 48], [0, 90.0, 36], [0, 0, 1]])
    Ki = np.linalg.inv(K)
    u, v = np.meshgrid(np.arange(w) + 0.5, np.arange(h) + 0.5)
    ray = np.stack([u, v, np.ones_like(u)], -1) @ Ki.T
    n = np.array([0.1, -0.3, -1.0])
    n /= np.linalg.norm(n)
    xs = [-2.0, -1.0, 0.0, 1.0, 2.0]
    deps, Rs, ts = [], [], []
    for x in xs:
        a = 0.02 * x
        R = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
        t = -R @ np.array([x, 0.3 * x, 0.0])
        C = -R.T @ t
        dirw = ray @ R
        s = -(n @ C + 40.0) / (dirw @ n)
        d = s * (1 + noise * rng.standard_normal(s.shape))
        d[rng.random(d.shape) < 0.05] = 0.0           # holes
        deps.append(d.astype(np.float32))
        Rs.append(R)
        ts.append(t)
    return K, deps, Rs, ts


@pytest.mark.parametrize("noise", [0.0, 0.05, 0.2])
def test_geometric_filter_matches_oracle(orc, hd, noise):
    rng = np.random.default_rng(int(noise * 100))
    K, deps, Rs, ts = _plane_maps(rng, noise)
    ref = 2
    nb = [0, 1, 3, 4]
    Rr = np.array([Rs[k] @ Rs[ref].T for k in nb])
    tr = np.array([ts[k] - Rs[k] @ Rs[ref].T @ ts[ref] for k in nb])
    hits_e, keep_e = orc.geo_consistency(K, deps[ref], [deps[k] for k in nb], Rr, tr, 10.0, 3)
    dref = hd.upload(deps[ref])
    hits, keep = hd.filter_geometric(K, dref, [hd.upload(deps[k]) for k in nb], Rr, tr, 10.0, 3)
    assert np.array_equal(hits.numpy(), hits_e), np.mean(hits.numpy() == hits_e)
    assert np.array_equal(keep.numpy(), keep_e), np.mean(keep.numpy() == keep_e)
    assert np.array_equal(dref.numpy() > 0, keep.numpy().astype(bool))
    if noise == 0.0:
        assert keep_e.mean() > 0.5


def test_frame_with_dog_filter(orc, fm):
    wl = scenegen.make_workload("config2_small")
    wl = dict(wl, params=dict(wl["params"], dog_filter=1))
    ref = orc.run_frame(wl)
    mask = orc.dog_mask(wl["ref"]["img"]).astype(bool)
    cfg = fm.config_from_params(wl["params"], keep_levels=1)
    with fm.Handle(cfg) as h:
        out = h.run_frame(wl)
        lab = h.level_map(0, 4)
    d = out["depth"]
    assert np.all(d[~mask] == 0) and np.all(out["conf"][~mask] == 0) and np.all(out["normal"][~mask] == 0)
    assert np.all(ref["depth"][~mask] == 0)
    agree = lab == orc.run_frame(wl, keep=True)["levels"][0]["label"]
    ok = mask & agree & (ref["depth"] > 0)
    assert np.max(np.abs(d[ok] - ref["depth"][ok]) / ref["depth"][ok]) <= 1e-3
