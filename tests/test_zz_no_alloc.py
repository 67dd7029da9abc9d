"""The allocation-free DoG filter (its scratch in the library's static device
array) against the allocating entry point, through the C ABI: two calls in a
row, the second on a smaller image, must give the same mask and the same
invalidated maps; an image above the array's limit is rejected."""
import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fm():
    import paper_2112_00821_amd as fm
    return fm


def _textured(h, w, seed):
    rng = np.random.default_rng(seed)
    img = np.full((h, w), 128, np.uint8)
    img[h // 8:h // 2, w // 8:w // 2] = rng.integers(0, 256, (h // 2 - h // 8, w // 2 - w // 8))
    img[h // 2:h - 4, w // 2:w - 4] = (rng.random((h - 4 - h // 2, w - 4 - w // 2)) * 6 + 125).astype(np.uint8)
    for i in range(60):
        y, x = rng.integers(0, h), rng.integers(0, w)
        img[y:y + 1 + i % 3, x:x + 1 + i % 4] = rng.integers(0, 256)
    return img


def _run(fm, hd, img, seed, noalloc):
    h, w = img.shape
    rng = np.random.default_rng(seed)
    depth = rng.random((h, w)).astype(np.float32) + 1
    normal = rng.random((h, w, 3)).astype(np.float32)
    conf = rng.random((h, w)).astype(np.float32)
    dd, nd, cd = hd.upload(depth), hd.upload(normal), hd.upload(conf)
    di = hd.upload(img)
    if noalloc:
        mask = hd.empty((h, w), np.uint8)
        hd.filter_dog_noalloc(di, dd, nd, cd, mask)
    else:
        mask = hd.filter_dog(di, dd, nd, cd)
    return mask.numpy(), dd.numpy(), nd.numpy(), cd.numpy()


def test_noalloc_dog_equals_allocating_filter_on_two_calls(fm):
    big = scenegen.make_workload("config2_small")["ref"]["img"]
    big = np.concatenate([big, _textured(*big.shape, 5)], axis=1)   # 640 x 184
    small = _textured(97, 131, 6)
    print(f"no-alloc DoG: {big.shape} then {small.shape}", flush=True)
    with fm.Handle() as hd:
        for img, seed in ((big, 1), (small, 2)):
            got = _run(fm, hd, img, seed, True)
            exp = _run(fm, hd, img, seed, False)
            for g, e, name in zip(got, exp, ("mask", "depth", "normal", "conf")):
                assert np.array_equal(g, e), (img.shape, name, np.mean(g != e))
            assert 0 < got[0].mean() < 1


def test_noalloc_dog_rejects_images_above_its_limit(fm):
    with fm.Handle() as hd:
        img = hd.upload(np.zeros((8, 8), np.uint8))
        st = fm.lib().fassmvs_filter_dog_noalloc(hd.h, img.vp, 4096, 1025, None, None, None, None)
        assert st == fm.EINVAL
        assert "maximum" in fm.lib().fassmvs_last_error(hd.h).decode()
