"""Forward parity of the HIP path (preprocess -> bin/sort -> raster) against the FP64 oracle.

Bit-exact: depth keys, per-primitive tile counts and the sorted (tile, primitive) lists.
Images: within 1e-4 per channel on every pixel without a knife-edge decision (a value within
1e-6 relative of a cutoff, or two contributors at equal depth), and few knife-edge pixels.
"""
import math

import numpy as np
import pytest
import torch

from drk_synth import Camera, Scene, config_c1, config_c2, intrinsics_hfov, scene_uniform_box
from oracle import drk_oracle as O
from tests._gpu_util import (IMG_TOL, KNIFE_MAX_FRAC, compare_image, compare_pixels, gpu_opts, log, need_gpu,
                             oracle_flat_lists, oracle_opts)

pytestmark = pytest.mark.gpu


def _ras(scene, cams, cap=1 << 20):
    from paper_2412_11752_amd import Rasterizer
    W = max(c.width for c in cams)
    H = max(c.height for c in cams)
    return Rasterizer(max(scene.n, 1), scene.K, W, H, max_views=len(cams), pair_capacity=cap)


def _u32(t):
    return t.cpu().numpy().view(np.uint32).astype(np.int64)


@pytest.fixture(scope="module")
def c1():
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene, cam = config_c1()
    log("c1: 64x64, 256 DRKs")
    ras = _ras(scene, [cam])
    ds = DRKScene.from_host(scene)
    rgb, T = ras.forward(ds, [cam], gpu_opts(counters=1))
    torch.cuda.synchronize()
    n_emit = ras.export("emitted").cpu().numpy()
    orc = O.render_image(scene, cam, oracle_opts())
    tiles, per, key = O.tile_lists(scene, cam, oracle_opts())
    return dict(scene=scene, cam=cam, ras=ras, ds=ds, rgb=rgb[0].cpu().numpy(), T=T[0].cpu().numpy(), orc=orc,
                tiles=tiles, per=per, key=key, n_emit=n_emit)


def test_c1_depth_keys_bit_exact(c1):
    gk = _u32(c1["ras"].export("depth_keys"))
    visible = np.array([len(c1["per"][j]) > 0 for j in range(c1["scene"].n)])
    assert visible.sum() > 50
    np.testing.assert_array_equal(gk[visible], c1["key"][visible].astype(np.int64))
    assert np.all(gk[~visible] == 0xFFFFFFFF)


def test_c1_tile_counts_bit_exact(c1):
    gc = _u32(c1["ras"].export("tile_counts"))
    oc = np.array([len(c1["per"][j]) for j in range(c1["scene"].n)])
    np.testing.assert_array_equal(gc, oc)


def test_c1_tile_lists_bit_exact(c1):
    ras = c1["ras"]
    gt = _u32(ras.export("pair_tiles"))
    gp = _u32(ras.export("pair_prims"))
    ot, op = oracle_flat_lists(c1["tiles"])
    assert gt.size == ot.size > 0
    np.testing.assert_array_equal(gt, ot)
    np.testing.assert_array_equal(gp, op)
    rng = _u32(ras.export("ranges")).reshape(-1, 2)
    for t in range(rng.shape[0]):
        s, e = rng[t]
        assert np.all(gt[s:e] == t)
        assert (e - s) == len(c1["tiles"].get(t, []))


def test_c1_image_parity(c1):
    H, W = c1["cam"].height, c1["cam"].width
    worst, nk, worst_k, err = compare_image(c1["rgb"], c1["orc"], H, W)
    log(f"c1 image: max err {worst:.3e} on unflagged pixels, {nk} knife-edge pixels (max {worst_k:.3e})")
    assert worst <= IMG_TOL
    assert nk <= max(2, KNIFE_MAX_FRAC * H * W)
    knife = c1["orc"].knife
    np.testing.assert_allclose(c1["T"].ravel()[~knife], c1["orc"].T[~knife], atol=IMG_TOL)
    ne = c1["n_emit"]
    np.testing.assert_array_equal(ne[~knife], c1["orc"].n_emit[~knife])
    assert c1["orc"].n_emit.max() >= 3


def test_c1_forward_is_deterministic(c1):
    """Repeated renders are bitwise equal, and the production launch (no per-pixel counters) gives the
    image of the instrumented one; the counter exports then report that they were not written."""
    from paper_2412_11752_amd._lib import DRK_EINVAL, DrkError
    ras, ds, cam = c1["ras"], c1["ds"], c1["cam"]
    a, Ta = ras.forward(ds, [cam], gpu_opts())
    b, Tb = ras.forward(ds, [cam], gpu_opts())
    assert torch.equal(a, b) and torch.equal(Ta, Tb)
    assert np.array_equal(a[0].cpu().numpy(), c1["rgb"])
    assert np.array_equal(Ta[0].cpu().numpy(), c1["T"])
    for what in ("emitted", "consumed", "contributors", "hits", "kernels"):
        with pytest.raises(DrkError) as e:
            ras.export(what)
        assert e.value.code == DRK_EINVAL


@pytest.mark.parametrize("cull_mode", [2])
def test_culling_changes_no_pixel(c1, cull_mode):
    """Sec. 4.4 culling only removes tiles the support cannot touch: binning every primitive to
    every tile gives the bitwise-identical image."""
    ras, ds, cam = c1["ras"], c1["ds"], c1["cam"]
    a, _ = ras.forward(ds, [cam], gpu_opts(cull_mode=cull_mode))
    assert np.array_equal(a[0].cpu().numpy(), c1["rgb"])


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 6, 7, 8])
def test_cache_lengths_match_oracle(c1, L):
    ras, ds, cam, scene = c1["ras"], c1["ds"], c1["cam"], c1["scene"]
    a, _ = ras.forward(ds, [cam], gpu_opts(cache_len=L))
    orc = O.render_image(scene, cam, oracle_opts(cache_len=L))
    worst, nk, _, _ = compare_image(a[0].cpu().numpy(), orc, cam.height, cam.width)
    log(f"cache_len={L}: max err {worst:.3e}, knife {nk}")
    assert worst <= IMG_TOL


def test_no_lowpass_matches_oracle(c1):
    ras, ds, cam, scene = c1["ras"], c1["ds"], c1["cam"], c1["scene"]
    a, _ = ras.forward(ds, [cam], gpu_opts(lowpass=False))
    orc = O.render_image(scene, cam, oracle_opts(lowpass=False))
    worst, nk, _, _ = compare_image(a[0].cpu().numpy(), orc, cam.height, cam.width)
    assert worst <= IMG_TOL


@pytest.mark.parametrize("alpha_min,alpha_max,T_min,near,lowpass", [
    (0.05, 0.6, 0.05, 0.2, True),       # tight supports, strong clamp, early stop
    (1e-3, 0.999, 1e-5, 0.2, True),     # wide supports
    (1e-3, 0.999, 1e-5, 3.6, False),    # near plane through the back half of the scene
    (0.02, 0.9, 0.3, 3.0, True),        # near plane at the front face, stop at T < 0.3
])
def test_other_thresholds_match_oracle(c1, alpha_min, alpha_max, T_min, near, lowpass):
    """The cutoffs the compositing takes as options (alpha_min, the alpha clamp, the transmittance
    stop, the near plane; Sec. 4.4) set from the caller rather than their defaults: the image, the
    per-DRK tile counts and the tile lists match the oracle run with the same values."""
    from paper_2412_11752_amd import make_opts
    ras, ds, cam, scene = c1["ras"], c1["ds"], c1["cam"], c1["scene"]
    sl = math.sqrt(0.5) if lowpass else 0.0
    a, _ = ras.forward(ds, [cam], make_opts(alpha_min=alpha_min, alpha_max=alpha_max, T_min=T_min, near=near,
                                            lowpass_sl=sl))
    oo = O.Opts(alpha_min=alpha_min, alpha_max=alpha_max, T_min=T_min, near=near, lowpass_sl=sl).f32()
    orc = O.render_image(scene, cam, oo)
    worst, nk, _, _ = compare_image(a[0].cpu().numpy(), orc, cam.height, cam.width)
    log(f"alpha_min {alpha_min} alpha_max {alpha_max} T_min {T_min} near {near} lowpass {lowpass}: "
        f"max err {worst:.2e}, knife {nk}")
    assert worst <= IMG_TOL
    tiles, per, _ = O.tile_lists(scene, cam, oo)
    assert np.array_equal(_u32(ras.export("tile_counts")), np.array([len(per[j]) for j in range(scene.n)], np.int64))
    ot, op = oracle_flat_lists(tiles)
    np.testing.assert_array_equal(_u32(ras.export("pair_tiles")), ot)
    np.testing.assert_array_equal(_u32(ras.export("pair_prims")), op)


def test_ragged_image_and_background():
    """An image that is not a multiple of the tile size, a non-zero background, SH colours."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    rng = np.random.default_rng(5)
    scene, _ = config_c2(n=2000)
    W, H = 53, 37
    from drk_synth import camera_lookat
    cam = camera_lookat((0.5, -3.5, 1.2), (0, 0, 0), (0, 0, 1), W, H, 60.0, bg=(0.2, 0.3, 0.4))
    ras = _ras(scene, [cam])
    rgb, T = ras.forward(DRKScene.from_host(scene), [cam], gpu_opts())
    orc = O.render_image(scene, cam, oracle_opts())
    worst, nk, _, _ = compare_image(rgb[0].cpu().numpy(), orc, H, W)
    log(f"ragged 53x37 SH3: max err {worst:.3e}, knife {nk}")
    assert worst <= IMG_TOL
    tiles, per, key = O.tile_lists(scene, cam, oracle_opts())
    ot, op = oracle_flat_lists(tiles)
    np.testing.assert_array_equal(_u32(ras.export("pair_tiles")), ot)
    np.testing.assert_array_equal(_u32(ras.export("pair_prims")), op)


def test_empty_and_fully_culled_scenes():
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene, cam = config_c1()
    cam2 = Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.R, cam.t, np.array([0.1, 0.2, 0.3], np.float32))
    empty = scene.subset(np.arange(0))
    ras = _ras(scene, [cam2])
    rgb, T = ras.forward(DRKScene.from_host(empty), [cam2], gpu_opts())
    assert torch.allclose(rgb[0], torch.tensor([0.1, 0.2, 0.3], device=rgb.device)[:, None, None].expand_as(rgb[0]))
    assert torch.all(T == 1)
    behind = Scene(scene.mu - np.array([[0], [0], [10]], np.float32), scene.q, scene.scale, scene.theta, scene.eta,
                   scene.tau, scene.opacity, scene.color, -1)
    rgb, T = ras.forward(DRKScene.from_host(behind), [cam2], gpu_opts())
    assert torch.all(T == 1)
    assert int(_u32(ras.export("tile_counts")).sum()) == 0


def test_pair_overflow_is_reported_and_recovered(c1):
    from paper_2412_11752_amd import Rasterizer
    from paper_2412_11752_amd._lib import DRK_EOVERFLOW
    scene, cam, ds = c1["scene"], c1["cam"], c1["ds"]
    ras = Rasterizer(scene.n, scene.K, cam.width, cam.height, pair_capacity=16, grow=False)
    ras.preprocess(ds, [cam], gpu_opts())
    ras.bin_sort()
    code, need = ras.status()
    assert code == DRK_EOVERFLOW and need == sum(len(v) for v in c1["tiles"].values())
    rgb, _ = ras.render_fwd()
    torch.cuda.synchronize()
    grow = Rasterizer(scene.n, scene.K, cam.width, cam.height, pair_capacity=16, grow=True)
    rgb, _ = grow.forward(ds, [cam], gpu_opts())
    assert np.array_equal(rgb[0].cpu().numpy(), c1["rgb"])


@pytest.mark.timeout(600)
def test_c2_sampled_pixels_and_tile_sample():
    """800x800, 100k DRKs on a sphere shell with SH3: 4096 seeded pixels against the oracle (which
    tests every primitive per pixel) and 200 seeded primitives' tile sets bit-exact."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene, cam = config_c2()
    log("c2: 800x800, 100k DRKs")
    ras = _ras(scene, [cam], cap=1 << 26)
    rgb, T = ras.forward(DRKScene.from_host(scene), [cam], gpu_opts())
    g = rgb[0].cpu().numpy()
    rng = np.random.default_rng(21)
    idx = rng.choice(cam.width * cam.height, 4096, replace=False)
    px, py = idx % cam.width, idx // cam.width
    orc = O.render_pixels(scene, cam, oracle_opts(), px, py)
    compare_pixels(g, orc, px, py, "c2 sampled", max_knife_frac=0.003)
    # tile sets of sampled primitives
    gt = _u32(ras.export("pair_tiles"))
    gp = _u32(ras.export("pair_prims"))
    keys = _u32(ras.export("depth_keys"))
    order = np.lexsort((gp, keys[gp], gt))
    assert np.array_equal(order, np.arange(gt.size))          # sorted by (tile, depth key, index)
    sample = rng.choice(scene.n, 200, replace=False)
    okey = O.centre_depth_f32(scene.mu, cam).view(np.uint32)
    for j in sample:
        ot = O.primitive_tiles(scene, cam, oracle_opts(), int(j))
        gtj = np.sort(gt[gp == j])
        assert np.array_equal(gtj, np.array(ot, np.int64)), j
        if ot:
            assert keys[j] == okey[j]


def _invalid_variants(scene):
    """Copies of the scene, each with primitive 5 made invalid in one way (the R19 reading)."""
    import copy
    K = scene.K
    out = {}

    def variant(name, fn):
        s = copy.deepcopy(scene)
        fn(s)
        out[name] = s
    variant("gap >= pi", lambda s: s.theta.__setitem__((slice(None), 5), np.linspace(0.0, 3.0, K, dtype=np.float32)))
    variant("zero scale", lambda s: s.scale.__setitem__((2, 5), 0.0))
    variant("negative scale", lambda s: s.scale.__setitem__((0, 5), -0.1))
    variant("nan centre", lambda s: s.mu.__setitem__((0, 5), np.nan))
    variant("inf quaternion", lambda s: s.q.__setitem__((1, 5), np.inf))
    variant("tau = 1", lambda s: s.tau.__setitem__(5, 1.0))
    variant("opacity 0", lambda s: s.opacity.__setitem__(5, 0.0))
    variant("eta > 1", lambda s: s.eta.__setitem__(5, 1.5))
    variant("angle >= 2 pi", lambda s: s.theta.__setitem__((K - 1, 5), np.float32(2 * np.pi)))
    return out


def test_validate_mode_reports_invalid_primitives(c1):
    """Invalid parameters (non-finite values, s <= 0, angles outside [0, 2 pi), a sector gap >= pi,
    o outside (0, 1], |tau| >= 1, eta outside [0, 1]): with validate set the frame reports DRK_EINVAL;
    without it the primitive is culled (no tiles, culled key) and the image matches the oracle's,
    which culls it too.  A valid scene passes validation."""
    from paper_2412_11752_amd import DRKScene
    from paper_2412_11752_amd._lib import DRK_EINVAL, DRK_OK
    scene, cam = c1["scene"], c1["cam"]
    ras = _ras(scene, [cam])
    assert O.primitive_valid(scene, 5)
    ras.preprocess(c1["ds"], [cam], _validate_opts(1))
    ras.bin_sort()
    assert ras.status()[0] == DRK_OK
    for name, bad in _invalid_variants(scene).items():
        assert not O.primitive_valid(bad, 5), name
        ds = DRKScene.from_host(bad)
        ras.preprocess(ds, [cam], _validate_opts(1))
        ras.bin_sort()
        code, _ = ras.status()
        assert code == DRK_EINVAL, name
        rgb, _ = ras.forward(ds, [cam], _validate_opts(0))
        assert ras.status()[0] == DRK_OK, name
        assert int(_u32(ras.export("tile_counts"))[5]) == 0, name
        assert int(_u32(ras.export("depth_keys"))[5]) == 0xFFFFFFFF, name
        orc = O.render_image(bad, cam, oracle_opts())
        worst, nk, _, _ = compare_image(rgb[0].cpu().numpy(), orc, cam.height, cam.width)
        log(f"invalid primitive ({name}): culled, image max err {worst:.2e}")
        assert worst <= IMG_TOL, name


def test_invalid_frame_arguments_are_refused(c1):
    """Options, cameras and scenes outside the accepted ranges give DRK_EINVAL from drk_preprocess,
    and a refused call leaves no frame behind: drk_bin_sort then refuses too, until a valid frame."""
    from paper_2412_11752_amd import DRKScene, make_opts
    from paper_2412_11752_amd._lib import DRK_EINVAL, DrkError
    ras, ds, cam, scene = c1["ras"], c1["ds"], c1["cam"], c1["scene"]

    def refused(d, cams, opts):
        with pytest.raises(DrkError) as e:
            ras.preprocess(d, cams, opts)
        assert e.value.code == DRK_EINVAL
        with pytest.raises(DrkError) as e:
            ras.bin_sort()
        assert e.value.code == DRK_EINVAL

    ras.preprocess(ds, [cam], gpu_opts())
    ras.bin_sort()
    for kw in (dict(alpha_min=0.0), dict(alpha_min=1.0), dict(alpha_max=0.0), dict(alpha_max=1.0),
               dict(T_min=0.0), dict(T_min=1.0), dict(near=0.0), dict(near=float("nan")), dict(lowpass_sl=-1.0),
               dict(cache_len=0), dict(cache_len=9), dict(cache_len=(1 << 30) - 1), dict(cull_mode=3),
               dict(key_mode=3), dict(launch_order=2), dict(counters=2)):
        refused(ds, [cam], make_opts(**kw))
    wide = Camera(cam.width + 1, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.R, cam.t)
    flat = Camera(cam.width, cam.height, 0.0, cam.fy, cam.cx, cam.cy, cam.R, cam.t)
    bad_r = Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, np.full((3, 3), np.nan, np.float32), cam.t)
    singular = Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, np.zeros((3, 3), np.float32), cam.t)
    for c in (wide, flat, bad_r, singular):
        refused(ds, [c], gpu_opts())
    refused(ds, [cam, cam], gpu_opts())                                   # more views than the workspace has
    refused(DRKScene.from_host(scene_uniform_box(1, scene.n + 1, K=8)), [cam], gpu_opts())
    refused(DRKScene.from_host(scene_uniform_box(1, 16, K=5)), [cam], gpu_opts())
    # a valid frame afterwards renders as before
    rgb, _ = ras.forward(ds, [cam], gpu_opts(counters=1))
    assert np.array_equal(rgb[0].cpu().numpy(), c1["rgb"])


def _validate_opts(v):
    from paper_2412_11752_amd import make_opts
    return make_opts(validate=v)


@pytest.mark.timeout(600)
def test_largest_image_three_pass_tile_sort():
    """8192x2176, the largest image the workspace accepts: 512 x 136 = 69632 tiles, so the tile ids
    take 17 bits and the pair sort three radix passes.  The whole sorted pair list is bit-exact
    against the oracle's tile lists and sampled pixels match the oracle."""
    need_gpu()
    from drk_synth import camera_lookat
    from paper_2412_11752_amd import DRKScene
    scene = scene_uniform_box(81, 400, K=8, half=1.0, s_lo=0.01, s_hi=0.06)
    cam = camera_lookat((0.0, 0.0, -3.0), (0, 0, 0), (0, 1, 0), 8192, 2176, 90.0, bg=(0.1, 0.0, 0.2))
    ras = _ras(scene, [cam], cap=1 << 22)
    rgb, _ = ras.forward(DRKScene.from_host(scene), [cam], gpu_opts())
    gt, gp = _u32(ras.export("pair_tiles")), _u32(ras.export("pair_prims"))
    tiles, _, _ = O.tile_lists(scene, cam, oracle_opts())
    ot, op = oracle_flat_lists(tiles)
    log(f"8192x2176: {gt.size} pairs, largest tile id {int(gt.max()) if gt.size else -1}")
    assert gt.size == ot.size > 0 and int(ot.max()) >= 65536
    np.testing.assert_array_equal(gt, ot)
    np.testing.assert_array_equal(gp, op)
    g = rgb[0].cpu().numpy()
    rng = np.random.default_rng(82)
    covered = np.unique(gt)
    ty, tx = covered // 512, covered % 512
    pick = rng.choice(covered.size, 256)
    px = tx[pick] * 16 + rng.integers(0, 16, 256)
    py = ty[pick] * 16 + rng.integers(0, 16, 256)
    px, py = np.concatenate([px, [8191, 0]]), np.concatenate([py, [2175, 2175]])
    orc = O.render_pixels(scene, cam, oracle_opts(), px, py)
    compare_pixels(g, orc, px, py, "8192x2176")


EXACT = 1 << 30


def test_exact_order_matches_oracle(c1):
    """cache_len >= 2^30: every contribution composited by hit depth (Sec. 4.4 Cache Sorting's ideal
    order), against the oracle's exact mode, on the 64x64 scene and on a dense 96x80 scene of
    intersecting primitives where the 8-slot cache gives a different image."""
    from paper_2412_11752_amd import DRKScene
    ras, ds, cam, scene = c1["ras"], c1["ds"], c1["cam"], c1["scene"]
    a, T = ras.forward(ds, [cam], gpu_opts(cache_len=EXACT))
    orc = O.render_image(scene, cam, oracle_opts(cache_len=O.EXACT))
    worst, nk, _, _ = compare_image(a[0].cpu().numpy(), orc, cam.height, cam.width)
    log(f"exact order 64x64: max err {worst:.2e}, knife {nk}")
    assert worst <= IMG_TOL
    np.testing.assert_allclose(T[0].cpu().numpy().ravel()[~orc.knife], orc.T[~orc.knife], atol=IMG_TOL)
    from drk_synth import camera_lookat
    dense = scene_uniform_box(44, 1500, K=8, half=0.7, s_lo=0.05, s_hi=0.35)
    cam2 = camera_lookat((0.3, -0.2, -3.0), (0, 0, 0), (0, 1, 0), 96, 80, 60.0, bg=(0.1, 0.2, 0.3))
    r2 = _ras(dense, [cam2])
    d2 = DRKScene.from_host(dense)
    ex, _ = r2.forward(d2, [cam2], gpu_opts(cache_len=EXACT))
    c8, _ = r2.forward(d2, [cam2], gpu_opts(cache_len=8))
    oe = O.render_image(dense, cam2, oracle_opts(cache_len=O.EXACT))
    o8 = O.render_image(dense, cam2, oracle_opts(cache_len=8))
    we, nke, _, _ = compare_image(ex[0].cpu().numpy(), oe, cam2.height, cam2.width)
    w8, nk8, _, _ = compare_image(c8[0].cpu().numpy(), o8, cam2.height, cam2.width)
    gap = float(np.abs(oe.rgb - o8.rgb).max())
    log(f"exact order 96x80 dense: max err {we:.2e} (knife {nke}); cache-8 {w8:.2e} (knife {nk8}); "
        f"exact vs cache-8 differ by up to {gap:.3f}")
    assert we <= IMG_TOL and w8 <= IMG_TOL
    assert gap > 1e-3 and float((ex - c8).abs().max()) > 1e-3


def test_exact_order_equals_cache_on_fronto_parallel_planes():
    """Every plane parallel to the image: the centre-depth pre-sort is already the hit-depth order, so
    the cache emits in exact order and both images are bitwise equal (the fronto-parallel pin)."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene = scene_uniform_box(45, 600, K=8, half=0.8, s_lo=0.05, s_hi=0.3)
    scene.q[:] = 0.0
    scene.q[0] = 1.0
    fx, fy, cx, cy = intrinsics_hfov(80, 64, 60.0)
    cam = Camera(80, 64, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.array([0, 0, 3.0], np.float32),
                 np.array([0.1, 0.1, 0.1], np.float32))
    ras = _ras(scene, [cam])
    ds = DRKScene.from_host(scene)
    ex, Te = ras.forward(ds, [cam], gpu_opts(cache_len=EXACT))
    c8, T8 = ras.forward(ds, [cam], gpu_opts(cache_len=8))
    assert torch.equal(ex, c8) and torch.equal(Te, T8)
    orc = O.render_image(scene, cam, oracle_opts(cache_len=O.EXACT))
    worst, nk, _, _ = compare_image(ex[0].cpu().numpy(), orc, cam.height, cam.width)
    assert worst <= IMG_TOL


def test_exact_order_refuses_other_outputs(c1):
    from paper_2412_11752_amd._lib import DRK_EINVAL, DrkError
    ras, ds, cam = c1["ras"], c1["ds"], c1["cam"]
    ras.preprocess(ds, [cam], gpu_opts(cache_len=EXACT))
    ras.bin_sort()
    for call in (lambda: ras.render_trace(8), lambda: ras.render_depth_normal()):
        with pytest.raises(DrkError) as e:
            call()
        assert e.value.code == DRK_EINVAL
