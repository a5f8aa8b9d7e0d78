"""Forward parity beyond the 64x64 case: other K, several views in one call, primitives that cross
the near plane, and the 1M-DRK 1080p and 3M-DRK eight-view workloads at full size (sampled pixels
against the FP64 oracle, sampled primitives' tile sets and depth keys bit-exact)."""
import math

import numpy as np
import pytest
import torch

from drk_synth import (Camera, Scene, camera_lookat, config_c3, config_c5, draw_angles, intrinsics_hfov,
                       scene_sphere_shell, scene_uniform_box)
from oracle import drk_oracle as O
from tests._gpu_util import IMG_TOL, compare_image, compare_pixels, gpu_opts, log, need_gpu, oracle_opts

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32).astype(np.int64)


def _rasterizer(scene, cams, cap):
    from paper_2412_11752_amd import Rasterizer
    return Rasterizer(scene.n, scene.K, max(c.width for c in cams), max(c.height for c in cams),
                      max_views=len(cams), pair_capacity=cap)


def _views(rgb_flat, cams):
    out, off = [], 0
    g = rgb_flat.reshape(-1).cpu().numpy()
    for c in cams:
        n = c.width * c.height
        out.append(g[3 * off:3 * (off + n)].reshape(3, c.height, c.width))
        off += n
    return out


@pytest.mark.parametrize("K", [3, 5, 16])
def test_other_basis_counts_match_oracle(K):
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene = scene_uniform_box(40 + K, 1500, K=K)
    cam = camera_lookat((0.3, -0.2, -3.2), (0, 0, 0), (0, 1, 0), 96, 80, 60.0, bg=(0.1, 0.2, 0.3))
    ras = _rasterizer(scene, [cam], 1 << 20)
    rgb, _ = ras.forward(DRKScene.from_host(scene), [cam], gpu_opts())
    orc = O.render_image(scene, cam, oracle_opts())
    worst, nk, _, _ = compare_image(rgb[0].cpu().numpy(), orc, cam.height, cam.width)
    log(f"K={K}: max err {worst:.2e}, knife {nk}")
    assert worst <= IMG_TOL and nk <= 8


def test_views_of_different_sizes_in_one_call():
    """Three views of different sizes share one preprocess/bin/raster call; each matches the oracle
    and the tile lists of each view are sorted by (tile, depth key, index)."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene = scene_uniform_box(9, 2500, K=8)
    cams = [camera_lookat((0, 0, -3.0), (0, 0, 0), (0, 1, 0), 64, 48, 60.0),
            camera_lookat((2.5, 0.5, -1.5), (0, 0, 0), (0, 1, 0), 50, 70, 70.0, bg=(0.2, 0.2, 0.2)),
            camera_lookat((-1.0, 2.8, 0.5), (0, 0, 0), (0, 0, 1), 33, 17, 50.0)]
    ras = _rasterizer(scene, cams, 1 << 20)
    rgb, _ = ras.forward(DRKScene.from_host(scene), cams, gpu_opts())
    for v, (g, cam) in enumerate(zip(_views(rgb, cams), cams)):
        orc = O.render_image(scene, cam, oracle_opts())
        worst, nk, _, _ = compare_image(g, orc, cam.height, cam.width)
        log(f"view {v} {cam.width}x{cam.height}: max err {worst:.2e}, knife {nk}")
        assert worst <= IMG_TOL and nk <= 4
        gt, gp = _u32(ras.export("pair_tiles", v)), _u32(ras.export("pair_prims", v))
        keys = _u32(ras.export("depth_keys", v))
        assert np.array_equal(np.lexsort((gp, keys[gp], gt)), np.arange(gt.size))
        tiles, _, _ = O.tile_lists(scene, cam, oracle_opts())
        ot, op = [], []
        for t in sorted(tiles):
            for _, j in tiles[t]:
                ot.append(t)
                op.append(j)
        assert np.array_equal(gt, np.array(ot)) and np.array_equal(gp, np.array(op))


def _tiny_views():
    """A view smaller than two tiles, one pixel, one row, one column and a view inside one tile."""
    return [camera_lookat((0.3, -3.2, 1.0), (0, 0, 0), (0, 0, 1), 40, 24, 60.0, bg=(0.1, 0.2, 0.3)),
            camera_lookat((2.5, 1.0, 1.5), (0, 0, 0), (0, 0, 1), 1, 1, 20.0),
            camera_lookat((-2.0, 2.5, 0.5), (0, 0, 0), (0, 0, 1), 37, 1, 60.0),
            camera_lookat((0.0, 0.5, -3.5), (0, 0, 0), (0, 1, 0), 1, 29, 60.0),
            camera_lookat((-3.0, -1.0, -1.0), (0, 0, 0), (0, 0, 1), 7, 5, 45.0, bg=(1.0, 1.0, 1.0))]


@pytest.mark.parametrize("sh_degree", [0, 1, 2])
def test_lower_sh_degrees_on_degenerate_views(sh_degree):
    """SH colour of degree 0, 1 and 2 (Sec. 3.1; the other tests use plain RGB or degree 3), on
    views of one pixel, one row, one column and less than a tile, all in one call: images within
    the tolerance of the oracle, tile lists bit-exact."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene = scene_sphere_shell(21 + sh_degree, 1500, K=8, sh_degree=sh_degree)
    assert scene.color.shape[0] == 3 * (sh_degree + 1) ** 2
    cams = _tiny_views()
    ras = _rasterizer(scene, cams, 1 << 20)
    rgb, _ = ras.forward(DRKScene.from_host(scene), cams, gpu_opts())
    for v, (g, cam) in enumerate(zip(_views(rgb, cams), cams)):
        orc = O.render_image(scene, cam, oracle_opts())
        worst, nk, _, _ = compare_image(g, orc, cam.height, cam.width)
        log(f"SH{sh_degree} view {v} {cam.width}x{cam.height}: max err {worst:.2e}, knife {nk}, "
            f"emitted {int(orc.n_emit.sum())}")
        assert worst <= IMG_TOL
        tiles, _, _ = O.tile_lists(scene, cam, oracle_opts())
        ot = [t for t in sorted(tiles) for _ in tiles[t]]
        op = [j for t in sorted(tiles) for _, j in tiles[t]]
        assert np.array_equal(_u32(ras.export("pair_tiles", v)), np.array(ot, np.int64))
        assert np.array_equal(_u32(ras.export("pair_prims", v)), np.array(op, np.int64))


def _extreme_scene(seed=31, n=600, K=8):
    """Valid parameters at the ends of their ranges, cycled over the primitives: eta 0 (pure L2) and
    1 (pure L1), tau -0.99 and 0.99, opacity 1, 0.999 and just above the 1/255 cutoff, one basis 100x
    shorter than the rest, and sectors of 1e-3 rad next to a 3.1 rad one (widest gap below pi)."""
    base = scene_uniform_box(seed, n, K=K, s_lo=0.05, s_hi=0.4)
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    eta = np.choose(i % 3, [np.zeros(n), np.ones(n), base.eta]).astype(np.float32)
    tau = np.choose(i % 4, [np.full(n, -0.99), np.full(n, 0.99), np.zeros(n), base.tau]).astype(np.float32)
    o = np.choose(i % 5, [np.ones(n), np.full(n, 0.999), np.full(n, 0.0045), np.full(n, 0.5),
                          base.opacity]).astype(np.float32)
    s = base.scale.copy()
    s[0, ::3] *= 0.01
    th = base.theta.astype(np.float64)
    rest = 3.101 + (2 * math.pi - 3.101) * np.arange(1, K - 2) / (K - 2)
    for j in range(0, n, 2):
        ang = np.concatenate([[0.0, 1e-3, 3.101], rest]) + rng.uniform(0, 2 * math.pi)
        th[:, j] = np.sort(np.mod(ang, 2 * math.pi))
    th = np.minimum(th, np.nextafter(np.float32(2 * math.pi), np.float32(0))).astype(np.float32)
    return Scene(base.mu, base.q, s, th, eta, tau, o, base.color, -1)


@pytest.mark.parametrize("lowpass", [True, False])
def test_extreme_valid_parameters_match_oracle(lowpass):
    """Primitives at the ends of the valid parameter ranges pass validation, and their image, tile
    counts and tile lists match the oracle's."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene, make_opts
    from paper_2412_11752_amd._lib import DRK_OK
    scene = _extreme_scene()
    assert all(O.primitive_valid(scene, j) for j in range(scene.n))
    cam = camera_lookat((0.4, -0.3, -3.4), (0, 0, 0), (0, 1, 0), 72, 56, 60.0, bg=(0.05, 0.1, 0.15))
    ras = _rasterizer(scene, [cam], 1 << 20)
    ds = DRKScene.from_host(scene)
    ras.preprocess(ds, [cam], make_opts(validate=1, lowpass_sl=math.sqrt(0.5) if lowpass else 0.0))
    ras.bin_sort()
    assert ras.status()[0] == DRK_OK
    rgb, _ = ras.forward(ds, [cam], gpu_opts(lowpass=lowpass))
    orc = O.render_image(scene, cam, oracle_opts(lowpass=lowpass))
    worst, nk, _, _ = compare_image(rgb[0].cpu().numpy(), orc, cam.height, cam.width)
    log(f"extreme parameters, lowpass {lowpass}: max err {worst:.2e}, knife {nk}, emitted {int(orc.n_emit.sum())}")
    assert worst <= IMG_TOL
    tiles, per, _ = O.tile_lists(scene, cam, oracle_opts(lowpass=lowpass))
    assert np.array_equal(_u32(ras.export("tile_counts")), np.array([len(per[j]) for j in range(scene.n)]))
    ot = [t for t in sorted(tiles) for _ in tiles[t]]
    op = [j for t in sorted(tiles) for _, j in tiles[t]]
    assert np.array_equal(_u32(ras.export("pair_tiles")), np.array(ot, np.int64))
    assert np.array_equal(_u32(ras.export("pair_prims")), np.array(op, np.int64))


def _near_scene():
    rng = np.random.default_rng(13)
    n, K = 12, 8
    mu = rng.uniform(-0.5, 0.5, (3, n)).astype(np.float32)
    q = rng.normal(size=(4, n)).astype(np.float32)
    th = draw_angles(rng, K, n)
    s = np.exp(rng.uniform(math.log(0.15), math.log(0.6), (K, n))).astype(np.float32)
    col = rng.normal(0, 0.1, (48, n)).astype(np.float32)
    col[:3] = rng.uniform(0, 1, (3, n))
    return Scene(mu, q, s, th, rng.uniform(0, 1, n).astype(np.float32), rng.uniform(0, 0.9, n).astype(np.float32),
                 rng.uniform(0.3, 0.95, n).astype(np.float32), col, 3)


@pytest.mark.parametrize("lowpass", [False, True])
def test_primitives_crossing_the_near_plane(lowpass):
    """Large DRKs whose support crosses z = near: the clipped polygon, the hits behind the camera and
    the near cut must all agree with the oracle."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene = _near_scene()
    cams = []
    for z, W, H in ((2.5, 24, 24), (0.9, 80, 64), (0.45, 96, 96)):
        fx, fy, cx, cy = intrinsics_hfov(W, H, 60.0)
        cams.append(Camera(W, H, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.array([0, 0, z], np.float32),
                           np.array([0.2, 0.1, 0.0], np.float32)))
    for cam in cams:
        ras = _rasterizer(scene, [cam], 1 << 16)
        rgb, _ = ras.forward(DRKScene.from_host(scene), [cam], gpu_opts(lowpass=lowpass))
        orc = O.render_image(scene, cam, oracle_opts(lowpass=lowpass))
        worst, nk, _, _ = compare_image(rgb[0].cpu().numpy(), orc, cam.height, cam.width)
        log(f"near-plane scene, camera z={cam.t[2]:.2f} {cam.width}x{cam.height}: max err {worst:.2e}, knife {nk}")
        assert worst <= IMG_TOL and nk <= 4
        gc = _u32(ras.export("tile_counts"))
        oc = np.array([len(O.primitive_tiles(scene, cam, oracle_opts(lowpass=lowpass), j)) for j in range(scene.n)])
        assert np.array_equal(gc, oc)


def _sampled_check(scene, cam, g, prims, n_px, seed, label):
    rng = np.random.default_rng(seed)
    idx = rng.choice(cam.width * cam.height, n_px, replace=False)
    # plus the ragged last tile row and column
    idx = np.concatenate([idx, [cam.width * cam.height - 1, (cam.height - 1) * cam.width, cam.width - 1]])
    px, py = idx % cam.width, idx // cam.width
    orc = O.render_pixels(scene, cam, oracle_opts(), px, py, prims=prims)
    compare_pixels(g, orc, px, py, label)


def _tile_sample(ras, scene, cam, view, n, seed):
    gt, gp = _u32(ras.export("pair_tiles", view)), _u32(ras.export("pair_prims", view))
    keys = _u32(ras.export("depth_keys", view))
    assert np.array_equal(np.lexsort((gp, keys[gp], gt)), np.arange(gt.size))
    okey = O.centre_depth_f32(scene.mu, cam).view(np.uint32)
    listed = np.unique(gp)
    rng = np.random.default_rng(seed)
    for j in rng.choice(listed, min(n, listed.size), replace=False):
        ot = O.primitive_tiles(scene, cam, oracle_opts(), int(j))
        assert np.array_equal(np.sort(gt[gp == j]), np.array(ot, np.int64)), j
        assert keys[j] == okey[j]


@pytest.mark.timeout(600)
def test_headline_1m_1080p_sampled():
    """1M DRKs (K=8, SH3) at 1920x1080 from inside the cluster box, in the launch configuration the
    benchmark times: 4096 seeded pixels (and the image corners) against the oracle, 60 listed DRKs'
    tile sets and keys bit-exact."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene, cams = config_c3()
    cam = cams[3]
    ras = _rasterizer(scene, [cam], 6_000_000)
    rgb, _ = ras.forward(DRKScene.from_host(scene), [cam], gpu_opts())
    g = rgb[0].cpu().numpy()
    log("1M 1080p rendered")
    prims = O.Prims.from_scene(scene)
    _sampled_check(scene, cam, g, prims, 4096, 31, "1M 1080p")
    _tile_sample(ras, scene, cam, 0, 60, 32)


@pytest.mark.timeout(600)
def test_training_shape_1m_1297x840_sampled():
    """The same 1M-DRK scene at 1297x840 (81 x 53 tiles, ragged in both directions), the image size of
    the training-step workload, along its camera path: 4096 seeded pixels (and the image corners)
    against the oracle, 60 listed DRKs' tile sets and keys bit-exact."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene, cams = config_c3(width=1297, height=840)
    cam = cams[7]
    ras = _rasterizer(scene, [cam], 6_000_000)
    rgb, _ = ras.forward(DRKScene.from_host(scene), [cam], gpu_opts())
    g = rgb[0].cpu().numpy()
    log("1M 1297x840 rendered")
    prims = O.Prims.from_scene(scene)
    _sampled_check(scene, cam, g, prims, 4096, 41, "1M 1297x840")
    _tile_sample(ras, scene, cam, 0, 60, 42)


@pytest.mark.timeout(400)
def test_eight_views_3m_k16_sampled():
    """3M DRKs (K=16, SH3) in a 40-unit box, eight 1920x1080 views rendered in one call with
    per-view sort buffers: 24 seeded pixels in each of four views against the oracle, and 10 listed
    DRKs' tile sets in two views."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene, cams = config_c5()
    log("3M K=16 scene generated")
    ras = _rasterizer(scene, cams, 12_000_000)
    rgb, _ = ras.forward(DRKScene.from_host(scene), cams, gpu_opts())
    views = _views(rgb, cams)
    log(f"8 views rendered, pair capacity {ras.pair_capacity}")
    prims = O.Prims.from_scene(scene)
    for v in (0, 2, 5, 7):
        _sampled_check(scene, cams[v], views[v], prims, 24, 50 + v, f"3M K=16 view {v}")
    for v in (0, 5):
        _tile_sample(ras, scene, cams[v], v, 10, 60 + v)
    log(f"peak device memory {torch.cuda.max_memory_allocated() / 2**30:.2f} GiB (torch) + workspace "
        f"{ras.size_query(scene.n, scene.K, 1920, 1080, 8, ras.pair_capacity) / 2**30:.2f} GiB")


def test_launch_orders_give_identical_images():
    """Longest-tile-first and row-major launch orders change only which tile starts when: images,
    transmittance and per-pixel counters are bit-identical."""
    need_gpu()
    from drk_synth import config_c2
    from paper_2412_11752_amd import DRKScene, make_opts
    scene, cam = config_c2()
    ras = _rasterizer(scene, [cam], 1 << 23)
    ds = DRKScene.from_host(scene)
    out = []
    for order in (0, 1):
        rgb, T = ras.forward(ds, [cam], make_opts(launch_order=order, counters=1))
        out.append((rgb.clone(), T.clone(), ras.export("emitted").clone(), ras.export("consumed").clone()))
    log(f"800x800: launch orders compared over {out[0][0].numel()} values")
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("key_mode", ["centre", "nearest"])
def test_span_buffer_overflow_gives_the_same_lists(monkeypatch, key_mode):
    """A row-span buffer of 64 rows (DRK_SPAN_ROWS) leaves almost every primitive's spans unstored, so
    the duplication re-derives them from the scene: pairs, ranges, images and per-pixel counters are
    bit-identical to those of the default buffer."""
    need_gpu()
    from drk_synth import config_c2
    from paper_2412_11752_amd import DRKScene, make_opts
    scene, cam = config_c2()
    ds = DRKScene.from_host(scene)
    out = []
    for rows in (None, "64"):
        if rows is None:
            monkeypatch.delenv("DRK_SPAN_ROWS", raising=False)
        else:
            monkeypatch.setenv("DRK_SPAN_ROWS", rows)
        ras = _rasterizer(scene, [cam], 1 << 23)
        rgb, T = ras.forward(ds, [cam], make_opts(key_mode=key_mode, counters=1))
        out.append([rgb.clone(), T.clone()] + [ras.export(w).clone() for w in
                                                ("pair_tiles", "pair_prims", "ranges", "emitted", "consumed")])
        ras.close()
    log(f"800x800 {key_mode} keys: {out[0][2].numel()} pairs with the default and the 64-row span buffer")
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("cull_mode", [0, 1])
def test_large_primitives_full_lists_match_oracle(cull_mode):
    """Twelve DRKs a few hundred pixels wide at 256x256: most have more than 32 tiles, so their pairs
    come from the workgroup-per-primitive duplication.  The whole sorted pair list is bit-exact
    against the oracle's tile lists for the conservative polygon and the paper's endpoint polygon;
    the image is compared for the conservative one (the endpoint polygon can drop support, and the
    oracle's image evaluates every primitive at every pixel)."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene = _near_scene()
    fx, fy, cx, cy = intrinsics_hfov(256, 256, 60.0)
    cam = Camera(256, 256, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.array([0, 0, 2.5], np.float32),
                 np.array([0.2, 0.1, 0.0], np.float32))
    ras = _rasterizer(scene, [cam], 1 << 20)
    rgb, _ = ras.forward(DRKScene.from_host(scene), [cam], gpu_opts(cull_mode=cull_mode))
    counts = _u32(ras.export("tile_counts"))
    log(f"cull mode {cull_mode}: tiles per DRK {sorted(counts.tolist())}")
    assert (counts > 32).sum() >= 4
    gt, gp = _u32(ras.export("pair_tiles")), _u32(ras.export("pair_prims"))
    tiles, _, _ = O.tile_lists(scene, cam, oracle_opts(cull_mode=cull_mode))
    ot = [t for t in sorted(tiles) for _ in tiles[t]]
    op = [j for t in sorted(tiles) for _, j in tiles[t]]
    assert np.array_equal(gt, np.array(ot)) and np.array_equal(gp, np.array(op))
    if cull_mode != 0:
        return
    orc = O.render_image(scene, cam, oracle_opts())
    worst, nk, _, _ = compare_image(rgb[0].cpu().numpy(), orc, cam.height, cam.width)
    log(f"cull mode {cull_mode}: max err {worst:.2e}, knife {nk}")
    assert worst <= IMG_TOL and nk <= 8


def _frustum_edge_scene(seed, n, K, W, H, fx, fy, cx, cy):
    """DRKs centred near the four side planes of a camera at the origin looking along +z, from
    2 max_k s_k inside to 4 max_k s_k outside, in random orientations (a third nearly edge-on)."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(0.6, 5.0, n)
    side = rng.integers(0, 4, n)
    s = np.exp(rng.uniform(math.log(0.05), math.log(0.6), (K, n)))
    off = rng.uniform(-2.0, 4.0, n) * s.max(0)
    px = np.where(side == 0, 0.0, np.where(side == 1, float(W), rng.uniform(0, W, n)))
    py = np.where(side == 2, 0.0, np.where(side == 3, float(H), rng.uniform(0, H, n)))
    X = (px - cx) / fx * z + np.where(side == 0, -off, np.where(side == 1, off, 0.0))
    Y = (py - cy) / fy * z + np.where(side == 2, -off, np.where(side == 3, off, 0.0))
    mu = np.stack([X, Y, z]).astype(np.float32)
    q = rng.normal(size=(4, n))
    # a third nearly edge-on: a quarter turn about x (the normal leaves the view axis), then a turn
    # about the view axis, so that the tangent plane holds the view axis; slightly perturbed
    edge = rng.random(n) < 1 / 3
    a = rng.uniform(0, 2 * np.pi, n)
    h = math.sqrt(0.5)
    qe = np.stack([np.cos(a / 2) * h, np.cos(a / 2) * h, np.sin(a / 2) * h, np.sin(a / 2) * h])
    qe = qe + rng.normal(0, 0.01, (4, n))
    q = np.where(edge[None, :], qe, q).astype(np.float32)
    col = rng.normal(0, 0.1, (48, n)).astype(np.float32)
    col[:3] = rng.uniform(0, 1, (3, n))
    return Scene(mu, q, s.astype(np.float32), draw_angles(rng, K, n), rng.uniform(0, 1, n).astype(np.float32),
                 rng.uniform(0, 0.9, n).astype(np.float32), rng.uniform(0.05, 0.95, n).astype(np.float32), col, 3)


@pytest.mark.parametrize("cull_mode,lowpass", [(0, True), (0, False), (1, True), (1, False)])
def test_frustum_edge_primitives_keep_their_tiles(cull_mode, lowpass):
    """The frustum test before the polygon only drops DRKs that reach no pixel centre: for DRKs around
    the view's side planes, the GPU's per-DRK tile sets equal the oracle's, which has no frustum test
    (its polygon decides), for the conservative polygon and the paper's endpoint polygon."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    W, H, K, n = 160, 120, 8, 600
    fx, fy, cx, cy = intrinsics_hfov(W, H, 70.0)
    cam = Camera(W, H, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.zeros(3, np.float32),
                 np.array([0.1, 0.1, 0.1], np.float32))
    scene = _frustum_edge_scene(21 + cull_mode, n, K, W, H, fx, fy, cx, cy)
    ras = _rasterizer(scene, [cam], 1 << 18)
    ras.forward(DRKScene.from_host(scene), [cam], gpu_opts(cull_mode=cull_mode, lowpass=lowpass))
    gc = _u32(ras.export("tile_counts"))
    gt, gp = _u32(ras.export("pair_tiles")), _u32(ras.export("pair_prims"))
    g_sets = [set() for _ in range(n)]
    for t, j in zip(gt.tolist(), gp.tolist()):
        g_sets[j].add(t)
    oo = oracle_opts(cull_mode=cull_mode, lowpass=lowpass)
    o_sets = [set(O.primitive_tiles(scene, cam, oo, j)) for j in range(n)]
    oc = np.array([len(x) for x in o_sets])
    log(f"cull mode {cull_mode}, low-pass {lowpass}: {int((oc > 0).sum())} of {n} DRKs with tiles, "
        f"{int((oc == 0).sum())} without")
    assert (oc > 0).sum() >= n // 5 and (oc == 0).sum() >= n // 5
    assert np.array_equal(gc, oc)
    assert all(g == o for g, o in zip(g_sets, o_sets))


@pytest.mark.parametrize("cull_mode", [0, 1])
def test_many_small_primitives_thread_walk(cull_mode):
    """400k small DRKs (K = 8) seen whole at 1280x720: more than 131072 of them fit a 4-row window,
    so their polygons take the thread-per-DRK walk with the rows in registers.  Sampled DRKs' tile
    sets and depth keys are bit-exact against the oracle, and the lists are sorted.  With the paper's
    endpoint polygon the sample includes DRK 223537, whose polygon reaches one tile although the
    ball of radius sqrt(2) c max_k s_k around its centre lies outside the view (the frustum test
    must use that polygon's own radius)."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene = scene_uniform_box(77, 400_000, K=8, s_lo=0.002, s_hi=0.02)
    cam = camera_lookat((0.0, 0.3, -2.6), (0, 0, 0), (0, 1, 0), 1280, 720, 60.0)
    ras = _rasterizer(scene, [cam], 1 << 23)
    ras.forward(DRKScene.from_host(scene), [cam], gpu_opts(cull_mode=cull_mode))
    gt, gp = _u32(ras.export("pair_tiles")), _u32(ras.export("pair_prims"))
    keys = _u32(ras.export("depth_keys"))
    gc = _u32(ras.export("tile_counts"))
    assert np.array_equal(np.lexsort((gp, keys[gp], gt)), np.arange(gt.size))
    okey = O.centre_depth_f32(scene.mu, cam).view(np.uint32)
    rng = np.random.default_rng(5 + cull_mode)
    listed = np.unique(gp)
    sample = list(rng.choice(listed, 300, replace=False)) + list(rng.choice(scene.n, 300, replace=False))
    if cull_mode == 1:
        sample.append(223537)
    oo = oracle_opts(cull_mode=cull_mode)
    log(f"cull mode {cull_mode}: {listed.size} DRKs listed, {gt.size} pairs")
    assert listed.size > 131072
    order = np.argsort(gp, kind="stable")
    starts = np.searchsorted(gp[order], np.arange(scene.n + 1))
    for j in sample:
        j = int(j)
        ot = O.primitive_tiles(scene, cam, oo, j)
        g = np.sort(gt[order[starts[j]:starts[j + 1]]])
        assert np.array_equal(g, np.array(ot, np.int64)), (j, g[:8], ot[:8])
        assert gc[j] == len(ot)
        if ot:
            assert keys[j] == okey[j]


@pytest.mark.parametrize("cull_mode,key_mode", [(0, 0), (1, 2)])
def test_polygon_paths_give_identical_lists(monkeypatch, cull_mode, key_mode):
    """The polygon kernels differ only in speed: the wave-per-DRK kernel (the default below 131072
    small DRKs), the thread-per-DRK walk (DRK_SMALL_MIN=0), the walk with DRKs admitted to the small
    list that then leave their 4-row window for the big list (DRK_WINDOW_ADMIT=16), and the walk with
    a 64-row span buffer (pools, and re-derivation in the duplication) give bitwise the same keys,
    counts, sorted pairs, ranges and image."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    scene = scene_uniform_box(23, 30000, K=8, s_lo=0.01, s_hi=0.25)
    cams = [camera_lookat((0.4, -0.3, -1.7), (0, 0, 0), (0, 1, 0), 640, 480, 75.0, bg=(0.1, 0.2, 0.3))]
    ds = DRKScene.from_host(scene)
    runs = {}
    for label, env in (("wave", {}), ("thread", {"DRK_SMALL_MIN": "0"}),
                       ("thread+leave", {"DRK_SMALL_MIN": "0", "DRK_WINDOW_ADMIT": "16"}),
                       ("thread+pools", {"DRK_SMALL_MIN": "0", "DRK_WINDOW_ADMIT": "16", "DRK_SPAN_ROWS": "64"})):
        for k in ("DRK_SMALL_MIN", "DRK_WINDOW_ADMIT", "DRK_SPAN_ROWS"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        ras = _rasterizer(scene, cams, 1 << 22)
        rgb, _ = ras.forward(ds, cams, gpu_opts(cull_mode=cull_mode, key_mode=key_mode))
        runs[label] = [rgb.cpu().numpy()] + [ras.export(w).cpu().numpy()
                                             for w in ("depth_keys", "tile_counts", "pair_tiles", "pair_prims", "ranges")]
        ras.close()
    counts = runs["wave"][2].view(np.uint32)
    log(f"cull mode {cull_mode}, key mode {key_mode}: {int((counts > 0).sum())} DRKs with tiles, "
        f"{int(counts.astype(np.int64).sum())} pairs")
    for label in ("thread", "thread+leave", "thread+pools"):
        for a, b in zip(runs["wave"], runs[label]):
            assert np.array_equal(a, b), label
