"""Parametrization (raw -> activated parameters), its vector-Jacobian product and the Adam step
(supplement S4) of the HIP path against the FP64 oracle, and an activated scene rendered through
the forward path."""
import math

import numpy as np
import pytest
import torch

from drk_synth import Scene, camera_lookat
from oracle import drk_oracle as O
from tests._gpu_util import IMG_TOL, compare_image, gpu_opts, log, need_gpu, oracle_opts

pytestmark = pytest.mark.gpu


def _raw_host(n, K, seed, ncol=48):
    rng = np.random.default_rng(seed)
    f = lambda a: np.asarray(a, np.float32)
    return {"mu": f(rng.uniform(-1, 1, (3, n))), "q": f(rng.normal(size=(4, n))),
            "scale": f(rng.normal(-2.5, 0.7, (K, n))), "theta": f(rng.normal(0, 2, (K, n))),
            "eta": f(rng.normal(size=n)), "tau": f(rng.normal(size=n)), "opacity": f(rng.normal(1, 1, n)),
            "color": f(rng.normal(0, 0.3, (ncol, n)))}


def _to_dev(h, sh_degree):
    from paper_2412_11752_amd import DRKScene
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    return DRKScene(t(h["mu"]), t(h["q"]), t(h["scale"]), t(h["theta"]), t(h["eta"]), t(h["tau"]), t(h["opacity"]),
                    t(h["color"]), sh_degree)


def _oracle_raw(h):
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64))
    return {"mu": t(h["mu"].T), "q": t(h["q"].T), "scale": t(h["scale"].T), "theta": t(h["theta"].T),
            "eta": t(h["eta"]), "tau": t(h["tau"]), "opacity": t(h["opacity"]), "color": t(h["color"].T)}


FIELDS = ("mu", "q", "scale", "theta", "eta", "tau", "opacity", "color")


@pytest.mark.parametrize("K", [3, 8, 16])
def test_activation_matches_oracle(K):
    need_gpu()
    from paper_2412_11752_amd import activate
    h = _raw_host(20000, K, K)
    act = activate(_to_dev(h, 3))
    ref = O.activate(_oracle_raw(h))
    worst = {}
    for f in FIELDS:
        g = getattr(act, f).cpu().numpy().astype(np.float64)
        r = ref[f].numpy()
        r = r.T if r.ndim == 2 else r
        err = np.abs(g - r) / np.maximum(np.abs(r), 1.0)
        worst[f] = float(err.max())
    log(f"K={K}: {worst}")
    assert max(worst.values()) <= 2e-6
    th = act.theta.cpu().numpy().astype(np.float64)
    gaps = np.diff(np.concatenate([th, np.full((1, th.shape[1]), 2 * math.pi)], 0), axis=0)
    assert (th[0] == 0).all() and (gaps > 0).all() and (gaps < math.pi).all()


@pytest.mark.parametrize("K", [3, 8])
def test_activation_vjp_matches_oracle(K):
    need_gpu()
    from paper_2412_11752_amd import activate_bwd
    h = _raw_host(5000, K, 10 + K)
    rng = np.random.default_rng(20 + K)
    gh = {f: np.asarray(rng.normal(size=h[f].shape), np.float32) for f in FIELDS}
    g = activate_bwd(_to_dev(h, 3), _to_dev(gh, 3))
    ref = O.activate_vjp(_oracle_raw(h), _oracle_raw(gh))
    worst = {}
    for f in FIELDS:
        a = getattr(g, f).cpu().numpy().astype(np.float64)
        r = ref[f].numpy()
        r = r.T if r.ndim == 2 else r
        worst[f] = float((np.abs(a - r) / (np.abs(r).max() + 1e-30)).max())
    log(f"K={K}: {worst}")
    assert max(worst.values()) <= 1e-5


def test_adam_matches_oracle_over_three_steps():
    need_gpu()
    from paper_2412_11752_amd import adam_step
    n = 1_000_003
    rng = np.random.default_rng(5)
    p = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    P, M, V = (torch.as_tensor(a, device="cuda") for a in (p, m, v))
    rp, rm, rv = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in (1, 2, 3):
        g = rng.normal(0, 1e-2, n).astype(np.float32)
        adam_step(P, M, V, torch.as_tensor(g, device="cuda"), 5e-3, 0.9, 0.999, 1e-15, step)
        rp, rm, rv = O.adam_step(rp, rm, rv, g.astype(np.float64), 5e-3, 0.9, 0.999, 1e-15, step)
    err = float(np.abs(P.cpu().numpy() - rp).max())
    log(f"adam 3 steps over {n} elements: max |p - oracle| = {err:.2e}")
    assert err <= 2e-6
    assert np.allclose(M.cpu().numpy(), rm, rtol=1e-5, atol=1e-9)


def test_activated_scene_renders_like_oracle():
    """Raw parameters activated on the GPU are valid renderer inputs: the forward path renders them
    as the oracle renders the same (downloaded) parameters, and they equal the oracle's activation."""
    need_gpu()
    from paper_2412_11752_amd import Rasterizer, activate
    h = _raw_host(400, 8, 77, ncol=3)
    h["mu"] *= 0.8
    h["scale"] = np.asarray(h["scale"] + 0.6, np.float32)
    act = activate(_to_dev(h, -1))
    sc = Scene(*[getattr(act, f).cpu().numpy() for f in FIELDS], -1)
    ref = O.activate(_oracle_raw(h))
    np.testing.assert_allclose(sc.theta.astype(np.float64), ref["theta"].numpy().T, atol=2e-6)
    cam = camera_lookat((0.2, -0.1, -3.2), (0, 0, 0), (0, 1, 0), 64, 56, 60.0)
    ras = Rasterizer(400, 8, cam.width, cam.height, pair_capacity=1 << 18)
    rgb, _ = ras.forward(act, [cam], gpu_opts())
    orc = O.render_image(sc, cam, oracle_opts())
    worst, nk, _, _ = compare_image(rgb[0].cpu().numpy(), orc, cam.height, cam.width)
    log(f"activated scene: max err {worst:.2e}, knife {nk}")
    assert worst <= IMG_TOL and nk <= 30


def test_empty_inputs():
    need_gpu()
    from paper_2412_11752_amd import activate, adam_step
    h = _raw_host(0, 8, 1)
    a = activate(_to_dev(h, 3))
    assert a.n == 0
    z = torch.zeros(0, device="cuda")
    adam_step(z, z.clone(), z.clone(), z.clone(), 1e-3)
