"""The seeded synthetic inputs follow their stated recipes: sizes, parameter ranges and laws, valid
basis angles, camera placement, and the same arrays for the same seed.  CPU only."""
import math

import numpy as np
import pytest

from drk_synth import (c3_camera_path, config_c1, config_c2, config_c4_scenes, config_c5, draw_angles,
                       mesh_icosphere, mesh_scene, mesh_torus, scene_clusters, scene_uniform_box)


def _assert_common_laws(sc, s_lo, s_hi):
    n, K = sc.n, sc.K
    assert sc.q.shape == (4, n) and sc.scale.shape == (K, n) and sc.theta.shape == (K, n)
    np.testing.assert_allclose(np.linalg.norm(sc.q.astype(np.float64), axis=0), 1.0, atol=1e-6)
    assert sc.scale.min() >= np.float32(s_lo) * (1 - 1e-6) and sc.scale.max() <= np.float32(s_hi) * (1 + 1e-6)
    assert 0.0 <= sc.eta.min() and sc.eta.max() <= 1.0
    assert 0.0 <= sc.tau.min() and sc.tau.max() < 0.99
    assert 0.05 <= sc.opacity.min() and sc.opacity.max() <= 0.99
    th = sc.theta.astype(np.float64).T
    assert (th >= 0).all() and (th < 2 * math.pi).all() and (np.diff(th, axis=1) >= 0).all()
    gaps = np.diff(np.concatenate([th, th[:, :1] + 2 * math.pi], axis=1), axis=1)
    assert (gaps > 0).all() and (gaps < math.pi).all()
    # log-uniform scales: log s uniform, so its mean is the midpoint of [log s_lo, log s_hi]
    if n * K >= 2000:
        mid = 0.5 * (math.log(s_lo) + math.log(s_hi))
        assert abs(np.log(sc.scale.astype(np.float64)).mean() - mid) < 0.05 * (math.log(s_hi) - math.log(s_lo))


def test_c1_recipe():
    sc, cam = config_c1()
    assert (sc.n, sc.K, sc.sh_degree) == (256, 8, -1)
    assert np.abs(sc.mu).max() <= 1.0
    _assert_common_laws(sc, 0.02, 0.3)
    assert sc.color.shape == (3, 256) and sc.color.min() >= 0 and sc.color.max() <= 1
    assert (cam.width, cam.height) == (64, 64) and np.all(cam.bg == 0)
    assert cam.fx == pytest.approx(32.0 / math.tan(math.radians(30.0)), rel=1e-6)
    np.testing.assert_allclose(cam.position(), [0.0, 0.0, -4.0], atol=1e-6)
    # the origin lies on the optical axis
    np.testing.assert_allclose(cam.R.astype(np.float64) @ np.zeros(3) + cam.t, [0.0, 0.0, 4.0], atol=1e-6)


def test_c2_recipe():
    sc, cam = config_c2(n=20_000)
    assert (sc.n, sc.K, sc.sh_degree) == (20_000, 8, 3)
    _assert_common_laws(sc, 0.02, 0.3)
    r = np.linalg.norm(sc.mu.astype(np.float64), axis=0)
    assert abs(r.mean() - 1.0) < 0.003 and 0.045 < r.std() < 0.055
    col = sc.color.reshape(16, 3, -1).astype(np.float64)
    assert col[0].min() >= 0 and col[0].max() <= 1
    assert abs(col[1:].mean()) < 0.002 and 0.048 < col[1:].std() < 0.052
    eye = cam.position()
    assert np.linalg.norm(eye) == pytest.approx(4.0, rel=1e-5)
    assert abs(math.degrees(math.asin(eye[2] / 4.0))) <= 30.0 + 1e-4
    # looks at the origin: it projects to the principal point
    pc = cam.R.astype(np.float64) @ np.zeros(3) + cam.t
    assert pc[2] > 0 and abs(pc[0] / pc[2]) < 1e-6 and abs(pc[1] / pc[2]) < 1e-6


def test_c3_camera_path_recipe():
    cams = c3_camera_path(202, 100, 1920, 1080, half=10.0)
    assert len(cams) == 100 and all((c.width, c.height) == (1920, 1080) for c in cams)
    pos = np.array([c.position() for c in cams])
    assert np.abs(pos).max() <= 8.0 + 1e-4
    fwd = np.array([c.R[2].astype(np.float64) for c in cams])
    step = np.linalg.norm(np.diff(pos, axis=0), axis=1)
    assert np.all(step <= 0.05 + 1e-5) and np.median(step) == pytest.approx(0.05, rel=1e-4)
    yaw = np.unwrap(np.arctan2(fwd[:, 1], fwd[:, 0]))
    np.testing.assert_allclose(np.diff(yaw), math.radians(1.0), atol=1e-5)
    pitch = np.degrees(np.arcsin(np.clip(fwd[:, 2], -1, 1)))
    assert np.abs(pitch).max() <= 30.0 + 1e-3


def test_cluster_scene_recipe():
    sc = scene_clusters(2, 100_000, K=8, half=10.0)
    assert (sc.n, sc.K, sc.sh_degree) == (100_000, 8, 3) and sc.color.shape == (48, 100_000)
    assert np.abs(sc.mu).max() <= 10.0
    _assert_common_laws(sc, 0.005, 0.5)
    # 64 clusters, not a uniform fill: the busiest tenth of an 8^3 grid of the box holds well over a
    # tenth of the centres (uniform centres: about 0.11)
    h, _ = np.histogramdd(sc.mu.T.astype(np.float64), bins=8, range=[(-10, 10)] * 3)
    busiest = np.sort(h.ravel())[::-1][:51]
    assert busiest.sum() / h.sum() > 0.3


def test_serving_scene_sizes():
    scenes = config_c4_scenes(n_scenes=3, lo=1000, hi=4000)
    assert [s.n for s in scenes] == [1000, 2000, 4000]
    assert all(s.K == 8 and s.sh_degree == 3 for s in scenes)


def test_c5_recipe():
    sc, cams = config_c5(n=30_000)
    assert (sc.K, sc.sh_degree) == (16, 3) and np.abs(sc.mu).max() <= 20.0
    _assert_common_laws(sc, 0.005, 0.5)
    path = c3_camera_path(404, 64, 1920, 1080, half=20.0)
    assert len(cams) == 8
    for c, p in zip(cams, path[::8]):
        np.testing.assert_array_equal(c.R, p.R)
        np.testing.assert_array_equal(c.t, p.t)


@pytest.mark.parametrize("K", [3, 4, 16])
def test_angles_are_valid_for_small_and_large_K(K):
    th = draw_angles(np.random.default_rng(K), K, 5000).astype(np.float64).T
    gaps = np.diff(np.concatenate([th, th[:, :1] + 2 * math.pi], axis=1), axis=1)
    assert (gaps > 0).all() and (gaps < math.pi).all() and (th < 2 * math.pi).all()


def test_generators_are_seeded():
    a, b, c = scene_uniform_box(5, 500), scene_uniform_box(5, 500), scene_uniform_box(6, 500)
    for f in ("mu", "q", "scale", "theta", "eta", "tau", "opacity", "color"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
        assert not np.array_equal(getattr(a, f), getattr(c, f))


def test_meshes():
    for level in (0, 1, 3):
        V, F = mesh_icosphere(level)
        assert F.shape == (20 * 4 ** level, 3) and V.shape[0] == 10 * 4 ** level + 2
        np.testing.assert_allclose(np.linalg.norm(V, axis=1), 1.0, atol=1e-12)
    V, F = mesh_torus(12, 6)
    assert F.shape == (72, 4) and V.shape == (72, 3)
    verts, faces, rgb = mesh_scene(5, 4, ico_level=1, torus=(8, 4))
    assert faces.shape[1] == 4 and rgb.shape == (faces.shape[0], 3)
    assert faces.min() >= -1 and faces.max() < verts.shape[0]
    tri = faces[:, 3] == -1
    assert tri.any() and (~tri).any() and (faces[:, :3] >= 0).all()
