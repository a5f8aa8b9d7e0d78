"""Per-tile pre-sort keys, front-to-back traces and the sorting-accuracy measures (supplement,
cache-sorting evaluation) of the HIP path against the FP64 oracle: tile lists and keys bit-exact,
images and composited sequences equal, and the metrics kernel equal to the oracle's measures of the
same traces."""

import numpy as np
import pytest
import torch

from drk_synth import camera_lookat, config_c3, scene_uniform_box
from oracle import drk_oracle as O
from tests._gpu_util import IMG_TOL, compare_image, gpu_opts, log, need_gpu, oracle_flat_lists, oracle_opts

pytestmark = pytest.mark.gpu

MODES = [1, 2]


def _u32(t):
    return t.cpu().numpy().view(np.uint32).astype(np.int64)


def _scene():
    """Large, randomly oriented kernels in a box: many overlaps per pixel, so the key order matters."""
    return scene_uniform_box(77, 600, K=8, half=1.0, s_lo=0.05, s_hi=0.5)


def _cam(W=80, H=72):
    return camera_lookat((0.4, -0.3, -3.0), (0, 0, 0), (0, 1, 0), W, H, 60.0, bg=(0.1, 0.1, 0.1))


def _render(scene, cam, opts, cap=64):
    from paper_2412_11752_amd import DRKScene, Rasterizer
    ras = Rasterizer(scene.n, scene.K, cam.width, cam.height, pair_capacity=1 << 20)
    ras.preprocess(DRKScene.from_host(scene), [cam], opts)
    ras.bin_sort()
    rgb, T, tn, ti, tz = ras.render_trace(cap)
    torch.cuda.synchronize()
    return ras, rgb, tn, ti, tz


@pytest.mark.parametrize("mode", MODES)
def test_tile_key_lists_and_keys_bit_exact(mode):
    need_gpu()
    scene, cam = _scene(), _cam()
    ras, *_ = _render(scene, cam, gpu_opts(key_mode=mode))
    gt, gp = _u32(ras.export("pair_tiles")), _u32(ras.export("pair_prims"))
    gk = _u32(ras.export("pair_keys"))
    tiles, _, _ = O.tile_lists(scene, cam, oracle_opts(key_mode=mode))
    ot, op = oracle_flat_lists(tiles)
    ok = np.array([k for t in sorted(tiles) for k, _ in tiles[t]], np.int64)
    log(f"key mode {mode}: {gt.size} pairs (oracle {ot.size}); keys equal {int((gk == ok).sum()) if gk.size == ok.size else 'n/a'}")
    assert np.array_equal(gt, ot) and np.array_equal(gp, op)
    assert np.array_equal(gk, ok)
    # lists ordered by (tile, key, index)
    assert np.array_equal(np.lexsort((gp, gk, gt)), np.arange(gt.size))


@pytest.mark.parametrize("mode", MODES)
def test_tile_keys_of_several_views_in_one_call(mode):
    """Three views of different sizes preprocessed and sorted in one call with per-tile keys: every
    view's lists, keys and image match the oracle's for that view alone."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene, Rasterizer
    scene = _scene()
    cams = [_cam(80, 72),
            camera_lookat((2.6, 0.4, -1.2), (0, 0, 0), (0, 1, 0), 45, 61, 70.0),
            camera_lookat((-0.8, 2.7, 0.9), (0, 0, 0), (0, 0, 1), 33, 17, 50.0, bg=(0.3, 0.2, 0.1))]
    ras = Rasterizer(scene.n, scene.K, 80, 72, max_views=len(cams), pair_capacity=1 << 20)
    rgb, _ = ras.forward(DRKScene.from_host(scene), cams, gpu_opts(key_mode=mode))
    flat = rgb.reshape(-1).cpu().numpy()
    off = 0
    for v, cam in enumerate(cams):
        npx = cam.width * cam.height
        g = flat[3 * off:3 * (off + npx)].reshape(3, cam.height, cam.width)
        off += npx
        gt, gp = _u32(ras.export("pair_tiles", v)), _u32(ras.export("pair_prims", v))
        gk = _u32(ras.export("pair_keys", v))
        tiles, _, _ = O.tile_lists(scene, cam, oracle_opts(key_mode=mode))
        ot, op = oracle_flat_lists(tiles)
        ok = np.array([k for t in sorted(tiles) for k, _ in tiles[t]], np.int64)
        assert np.array_equal(gt, ot) and np.array_equal(gp, op), v
        assert np.array_equal(gk, ok), v
        orc = O.render_image(scene, cam, oracle_opts(key_mode=mode))
        worst, nk, _, _ = compare_image(g, orc, cam.height, cam.width)
        log(f"key mode {mode}, view {v} {cam.width}x{cam.height}: {gt.size} pairs, max err {worst:.2e}, knife {nk}")
        assert worst <= IMG_TOL


@pytest.mark.parametrize("cache_len", [2, 3, 4, 5, 6, 7])
def test_every_cache_length_on_a_dense_scene(cache_len):
    """Cache lengths between 1 and 8 on the overlapping scene, where each length gives a different
    image (consecutive lengths differ by more than 0.16 somewhere): the image matches the oracle's."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene, Rasterizer
    scene, cam = _scene(), _cam()
    ras = Rasterizer(scene.n, scene.K, cam.width, cam.height, pair_capacity=1 << 20)
    rgb, _ = ras.forward(DRKScene.from_host(scene), [cam], gpu_opts(cache_len=cache_len))
    orc = O.render_image(scene, cam, oracle_opts(cache_len=cache_len))
    worst, nk, _, _ = compare_image(rgb[0].cpu().numpy(), orc, cam.height, cam.width)
    log(f"dense scene, cache_len={cache_len}: max err {worst:.2e}, knife {nk}")
    assert worst <= IMG_TOL


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("cache_len", [1, 8])
def test_images_and_traces_match_oracle(mode, cache_len):
    need_gpu()
    scene, cam = _scene(), _cam()
    ras, rgb, tn, ti, tz = _render(scene, cam, gpu_opts(key_mode=mode, cache_len=cache_len))
    orc = O.render_image(scene, cam, oracle_opts(key_mode=mode, cache_len=cache_len))
    H, W = cam.height, cam.width
    worst, nk, _, _ = compare_image(rgb.view(3, H, W).cpu().numpy(), orc, H, W)
    tn, ti, tz = tn.cpu().numpy(), ti.cpu().numpy(), tz.cpu().numpy()
    bad = 0
    zerr = 0.0
    for p in np.nonzero(~orc.knife)[0]:
        m = min(int(tn[p]), ti.shape[1])
        ref = orc.emitted[p]
        if int(tn[p]) != len(ref) or list(ti[p, :m]) != ref[:m]:
            bad += 1
            continue
        if m:
            zerr = max(zerr, float(np.max(np.abs(tz[p, :m] - np.array(orc.emitted_z[p][:m])) / np.array(orc.emitted_z[p][:m]))))
    log(f"key mode {mode}, L={cache_len}: image max err {worst:.2e}, knife {nk}, sequence mismatches {bad}, "
        f"max rel depth err {zerr:.2e}, mean composited {tn.mean():.1f}")
    assert worst <= IMG_TOL and nk <= H * W // 200
    assert bad == 0
    assert zerr <= 2e-5


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_trace_metrics_kernel_matches_oracle_measures(mode):
    """drk_trace_metrics on the recorded traces equals the oracle's measures of the same depth
    sequences (counts exactly, sums to float rounding), and the oracle's own traces give the same
    measures to within the few knife-edge pixels."""
    need_gpu()
    from paper_2412_11752_amd import trace_metrics
    scene, cam = _scene(), _cam()
    cap = 64
    _, _, tn, ti, tz = _render(scene, cam, gpu_opts(key_mode=mode, cache_len=4), cap)
    g = trace_metrics(tn, tz, cap)
    tnh, tzh = tn.cpu().numpy(), tz.cpu().numpy()
    seqs = [tzh[p, :min(int(tnh[p]), cap)] for p in range(tnh.size)]
    ref = O.sort_metrics(seqs)
    log(f"key mode {mode}: kernel {g}, oracle-on-trace {ref}")
    assert g["n"] == ref["n"] and g["pixels"] == ref["pixels"]
    assert g["truncated"] == int((tnh > cap).sum())
    assert g["accuracy"] == pytest.approx(ref["accuracy"], abs=1e-12)
    assert g["kendall_tau"] == pytest.approx(ref["kendall_tau"], rel=1e-9)
    assert g["mae"] == pytest.approx(ref["mae"], rel=1e-5)
    orc = O.render_image(scene, cam, oracle_opts(key_mode=mode, cache_len=4))
    full = O.sort_metrics(orc.emitted_z, cap=cap)
    log(f"oracle render: {full}")
    assert abs(full["accuracy"] - g["accuracy"]) <= 2e-3
    assert abs(full["kendall_tau"] - g["kendall_tau"]) <= 2e-3
    assert full["mae"] == pytest.approx(g["mae"], rel=1e-2)


def test_trace_of_empty_and_ragged_views():
    """Pixels with nothing to composite record n = 0; a view smaller than a tile works; cap 1
    keeps only the front entry."""
    need_gpu()
    scene = _scene()
    cam = _cam(13, 7)
    ras, rgb, tn, ti, tz = _render(scene, cam, gpu_opts(key_mode=2), cap=1)
    orc = O.render_image(scene, cam, oracle_opts(key_mode=2))
    tn, ti = tn.cpu().numpy(), ti.cpu().numpy()
    for p in np.nonzero(~orc.knife)[0]:
        assert int(tn[p]) == len(orc.emitted[p])
        if orc.emitted[p]:
            assert int(ti[p, 0]) == orc.emitted[p][0]
    far = camera_lookat((0.0, 0.0, -3.0), (0.0, 0.0, -10.0), (0, 1, 0), 20, 20, 60.0)
    _, _, tn2, _, _ = _render(scene, far, gpu_opts(key_mode=1))
    assert int(tn2.sum().item()) == 0


@pytest.mark.timeout(300)
def test_nearest_keys_at_1m_1080p_sampled():
    """1M DRKs at 1920x1080 with the nearest-distance key: 40 listed DRKs' tile sets and per-tile
    keys bit-exact, lists ordered by (tile, key, index), and 128 seeded pixels against the oracle."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene, Rasterizer
    scene, cams = config_c3()
    cam = cams[3]
    opts = gpu_opts(key_mode=2)
    oo = oracle_opts(key_mode=2)
    ras = Rasterizer(scene.n, scene.K, cam.width, cam.height, pair_capacity=6_000_000)
    rgb, _ = ras.forward(DRKScene.from_host(scene), [cam], opts)
    g = rgb[0].cpu().numpy()
    gt, gp, gk = _u32(ras.export("pair_tiles")), _u32(ras.export("pair_prims")), _u32(ras.export("pair_keys"))
    assert np.array_equal(np.lexsort((gp, gk, gt)), np.arange(gt.size))
    rng = np.random.default_rng(71)
    for j in rng.choice(np.unique(gp), 40, replace=False):
        sel = gp == j
        ot = O.primitive_tiles(scene, cam, oo, int(j))
        assert np.array_equal(np.sort(gt[sel]), np.array(ot, np.int64)), j
        kp = O.key_plane(scene, cam, oo, int(j))
        okeys = {t: O.tile_key(kp, cam, oo, t) for t in ot}
        assert all(int(k) == okeys[int(t)] for t, k in zip(gt[sel], gk[sel])), j
    idx = rng.choice(cam.width * cam.height, 128, replace=False)
    px, py = idx % cam.width, idx // cam.width
    orc = O.render_pixels(scene, cam, oo, px, py)
    err = np.abs(g[:, py, px].T.astype(np.float64) - orc.rgb).max(axis=1)
    log(f"1M 1080p nearest key: {gt.size} pairs, sampled max err {err[~orc.knife].max():.2e}, knife {int(orc.knife.sum())}")
    assert err[~orc.knife].max() <= IMG_TOL
