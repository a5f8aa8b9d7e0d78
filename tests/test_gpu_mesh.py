"""Mesh to DRK and the depth / normal channels (section "Converting Mesh to DRK" and its
supplement) of the HIP path against the FP64 oracle: converted parameters, rejected faces, and
colour, depth and normal images of converted meshes."""

import numpy as np
import pytest
import torch

from drk_synth import camera_lookat, config_c2, mesh_icosphere, mesh_scene
from oracle import drk_oracle as O
from tests._gpu_util import IMG_TOL, gpu_opts, log, need_gpu, oracle_opts

pytestmark = pytest.mark.gpu


def _gpu_mesh(V, F, C, K, tau=0.95, opacity=0.99):
    from paper_2412_11752_amd import mesh_to_drk
    dev = "cuda"
    v = torch.as_tensor(np.ascontiguousarray(V.T, np.float32), device=dev)
    f = torch.as_tensor(np.ascontiguousarray(F, np.int32), device=dev)
    c = torch.as_tensor(np.ascontiguousarray(np.asarray(C, np.float32).T), device=dev)
    return mesh_to_drk(v, f, c, K, tau, opacity)


def _host(ds):
    from drk_synth import Scene
    t = lambda a: a.cpu().numpy()
    return Scene(t(ds.mu), t(ds.q), t(ds.scale), t(ds.theta), t(ds.eta), t(ds.tau), t(ds.opacity), t(ds.color), -1)


def _rot(q):
    return O.quat_to_rotmat(torch.as_tensor(q.T.astype(np.float64))).numpy()


@pytest.mark.parametrize("K", [4, 8])
def test_mesh_conversion_matches_oracle(K):
    need_gpu()
    V, F, C = mesh_scene(5, n_instances=6, ico_level=3, torus=(32, 16))
    ds, rej = _gpu_mesh(V, F, C, K)
    g = _host(ds)
    o = O.mesh_to_drk(V, F, C, K=K)
    log(f"K={K}: {F.shape[0]} faces, rejected gpu {rej}, oracle {int((o.opacity == 0).sum())}")
    assert rej == int((o.opacity == 0).sum())
    assert np.array_equal(g.opacity == 0, o.opacity == 0)
    np.testing.assert_allclose(g.mu, o.mu, atol=1e-6)
    np.testing.assert_allclose(_rot(g.q), _rot(o.q), atol=2e-6)
    np.testing.assert_allclose(g.scale, o.scale, rtol=2e-6)
    np.testing.assert_allclose(g.theta, o.theta, atol=2e-6)
    assert np.array_equal(g.eta, o.eta) and np.array_equal(g.tau, o.tau) and np.array_equal(g.color, o.color)


def test_mesh_rejects_bad_faces():
    need_gpu()
    V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [2, 0, 0], [0.6, 0.4, 0]], float)
    F = np.array([[0, 1, 2, 3], [0, 1, 4, -1], [0, 1, 5, 2], [0, 3, 2, 1], [0, 1, 2, -1], [0, 1, 9, -1],
                  [0, 1, -1, -1]], np.int32)
    ds, rej = _gpu_mesh(V, F, np.ones((7, 3)), K=4)
    op = ds.opacity.cpu().numpy()
    log(f"opacity {op}, rejected {rej}")
    assert list(op > 0) == [True, False, False, True, True, False, False] and rej == 4


@pytest.mark.parametrize("mode", [0, 2])
def test_mesh_render_colour_depth_normal_match_oracle(mode):
    """A converted mesh scene (sharp faces, many overlaps) with the depth and normal channels; the
    nearest key matters most here (the supplement's remark on cache sorting for meshes)."""
    need_gpu()
    from paper_2412_11752_amd import Rasterizer
    V, F, C = mesh_scene(7, n_instances=4, ico_level=2, torus=(16, 8), half=0.8)
    ds, _ = _gpu_mesh(V, F, C, K=4, tau=0.9)
    host = _host(ds)
    cam = camera_lookat((0.3, 0.4, -3.2), (0, 0, 0), (0, 1, 0), 96, 80, 60.0, bg=(0.05, 0.05, 0.05))
    ras = Rasterizer(host.n, 4, cam.width, cam.height, pair_capacity=1 << 20)
    ras.preprocess(ds, [cam], gpu_opts(key_mode=mode))
    ras.bin_sort()
    rgb, T, depth, normal = ras.render_depth_normal()
    torch.cuda.synchronize()
    orc = O.render_image(host, cam, oracle_opts(key_mode=mode))
    H, W = cam.height, cam.width
    ok = ~orc.knife
    e_rgb = np.abs(rgb.view(3, H * W).cpu().numpy().T - orc.rgb).max(1)[ok].max()
    d = depth.cpu().numpy()
    e_d = (np.abs(d - orc.depth) / np.maximum(orc.depth, 1.0))[ok].max()
    e_n = np.abs(normal.view(3, H * W).cpu().numpy().T - orc.normal).max(1)[ok].max()
    e_T = np.abs(T.cpu().numpy() - orc.T)[ok].max()
    log(f"mesh scene {host.n} DRKs, key {mode}: rgb {e_rgb:.2e}, depth {e_d:.2e}, normal {e_n:.2e}, T {e_T:.2e}, "
        f"knife {int(orc.knife.sum())}, covered {(orc.T < 0.5).mean():.2f}")
    assert e_rgb <= IMG_TOL and e_n <= IMG_TOL and e_T <= IMG_TOL and e_d <= IMG_TOL
    assert orc.knife.sum() <= H * W // 100


def test_depth_normal_on_an_sh_scene():
    """The depth / normal variant leaves the colour bit-identical to the plain forward and matches
    the oracle's channels on sampled pixels of the 800x800 SH scene."""
    need_gpu()
    from paper_2412_11752_amd import DRKScene, Rasterizer
    scene, cam = config_c2()
    ras = Rasterizer(scene.n, scene.K, cam.width, cam.height, pair_capacity=1 << 23)
    ds = DRKScene.from_host(scene)
    rgb0, _ = ras.forward(ds, [cam], gpu_opts())
    rgb, T, depth, normal = ras.render_depth_normal()
    assert torch.equal(rgb0.reshape(-1), rgb)
    rng = np.random.default_rng(5)
    idx = rng.choice(cam.width * cam.height, 96, replace=False)
    px, py = idx % cam.width, idx // cam.width
    orc = O.render_pixels(scene, cam, oracle_opts(), px, py)
    ok = ~orc.knife
    d = depth.cpu().numpy()[idx]
    n = normal.view(3, -1).cpu().numpy()[:, idx].T
    e_d = (np.abs(d - orc.depth) / np.maximum(orc.depth, 1.0))[ok].max()
    e_n = np.abs(n - orc.normal).max(1)[ok].max()
    log(f"800x800 SH: depth {e_d:.2e}, normal {e_n:.2e}")
    assert e_d <= IMG_TOL and e_n <= IMG_TOL


@pytest.mark.timeout(300)
def test_icosphere_1m_faces_at_1080p_sampled():
    """1.3M-triangle icosphere converted on the GPU and rendered at 1920x1080 with depth and
    normals: 64 seeded pixels against the oracle (on the GPU-converted scene), and a converted
    sample of faces against the oracle's conversion."""
    need_gpu()
    from paper_2412_11752_amd import Rasterizer
    V, F = mesh_icosphere(8)
    V = V * 2.0
    F = np.concatenate([F, -np.ones((F.shape[0], 1), np.int32)], 1)
    rng = np.random.default_rng(3)
    C = rng.uniform(0.2, 1.0, (F.shape[0], 3)).astype(np.float32)
    ds, rej = _gpu_mesh(V, F, C, K=4, tau=0.9)
    assert rej == 0
    sel = rng.choice(F.shape[0], 200, replace=False)
    o = O.mesh_to_drk(V, F[sel], C[sel], K=4, tau=0.9)
    g = _host(ds).subset(sel)
    np.testing.assert_allclose(g.mu, o.mu, atol=1e-6)
    np.testing.assert_allclose(g.scale, o.scale, rtol=2e-6)
    cam = camera_lookat((0.5, 1.0, -5.0), (0, 0, 0), (0, 1, 0), 1920, 1080, 60.0)
    ras = Rasterizer(ds.n, 4, 1920, 1080, pair_capacity=8_000_000)
    ras.preprocess(ds, [cam], gpu_opts(key_mode=2))
    ras.bin_sort()
    code, need = ras.status()
    assert code == 0, need
    rgb, T, depth, normal = ras.render_depth_normal()
    idx = rng.choice(1920 * 1080, 64, replace=False)
    px, py = idx % 1920, idx // 1920
    host = _host(ds)
    orc = O.render_pixels(host, cam, oracle_opts(key_mode=2), px, py)
    ok = ~orc.knife
    e_rgb = np.abs(rgb.view(3, -1).cpu().numpy()[:, idx].T - orc.rgb).max(1)[ok].max()
    e_d = (np.abs(depth.cpu().numpy()[idx] - orc.depth) / np.maximum(orc.depth, 1.0))[ok].max()
    e_n = np.abs(normal.view(3, -1).cpu().numpy()[:, idx].T - orc.normal).max(1)[ok].max()
    log(f"icosphere 1.3M faces 1080p: pairs {ras.export('pair_tiles').numel()}, rgb {e_rgb:.2e}, depth {e_d:.2e}, "
        f"normal {e_n:.2e}, knife {int(orc.knife.sum())}")
    assert e_rgb <= IMG_TOL and e_d <= IMG_TOL and e_n <= IMG_TOL
