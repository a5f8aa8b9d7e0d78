"""Pins of the FP64 oracle against what the paper and mathematics fix (no GPU needed).

Each test names the passage it pins.  None of them re-types the oracle's own formula: they use
closed forms (2D Gaussian, isotropic Gaussian, L1 diamond), independent formulations (linear
solve for the ray-plane hit, heapq for the cache, scipy for spherical harmonics), invariants
(telescoping weights, Psi identities) and brute force on tiny inputs.
"""
import heapq
import math
import os

import numpy as np
import pytest
import torch

from drk_synth import Camera, Scene, config_c1, intrinsics_hfov
from oracle import drk_oracle as O

F64 = torch.float64
rng_global = np.random.default_rng(1234)


def _t(x):
    return torch.as_tensor(np.asarray(x, np.float64))


def _alpha(u, v, s, th, eta, tau, o):
    L = len(u)
    return O.drk_alpha_uv(_t(u), _t(v), _t(np.tile(s, (L, 1))), _t(np.tile(th, (L, 1))),
                          _t(np.full(L, eta)), _t(np.full(L, tau)), _t(np.full(L, o))).numpy()


# ---- Sec. 4.1, "2D Gaussian as a special case" (with the printed cos^2 -> sin^2 typo corrected)
def test_p1_gaussian_reduction():
    rng = np.random.default_rng(1)
    for _ in range(20):
        su, sv = rng.uniform(0.05, 2.0, 2)
        o = rng.uniform(0.1, 1.0)
        u, v = rng.normal(0, 1.5, (2, 500))
        a = _alpha(u, v, [su, sv, su, sv], [0, math.pi / 2, math.pi, 1.5 * math.pi], 0.0, 0.0, o)
        ref = o * np.exp(-0.5 * (u ** 2 / su ** 2 + v ** 2 / sv ** 2))   # Eq. (3), 2D-GS
        np.testing.assert_allclose(a, ref, rtol=1e-12, atol=1e-300)


# ---- Sec. 4.1: equal radial lengths give an isotropic Gaussian for any basis angles
def test_p2_equal_scales_isotropic():
    rng = np.random.default_rng(2)
    for K in (3, 5, 8, 16):
        th = np.sort(rng.uniform(0, 2 * math.pi, K))
        while np.max(np.diff(np.r_[th, th[0] + 2 * math.pi])) >= math.pi:
            th = np.sort(rng.uniform(0, 2 * math.pi, K))
        s = rng.uniform(0.1, 1.0)
        u, v = rng.normal(0, 1, (2, 400))
        a = _alpha(u, v, np.full(K, s), th, 0.0, 0.0, 1.0)
        np.testing.assert_allclose(a, np.exp(-(u * u + v * v) / (2 * s * s)), rtol=1e-12)


# ---- Sec. 4.2: with eta = 1, equal lengths and axis bases the unit L1 ball is the diamond
def test_p3_l1_diamond():
    rng = np.random.default_rng(3)
    s = 0.7
    u, v = rng.normal(0, 1, (2, 400))
    a = _alpha(u, v, np.full(4, s), [0, math.pi / 2, math.pi, 1.5 * math.pi], 1.0, 0.0, 1.0)
    np.testing.assert_allclose(a, np.exp(-0.5 * ((np.abs(u) + np.abs(v)) / s) ** 2), rtol=1e-12)


# ---- Sec. 4.2, Eq. (L1): the L1 level set through the endpoints is the straight segment e_k e_{k+1};
# a point lam*e_k + mu*e_{k+1} (lam, mu >= 0) has r1 = lam + mu, for arbitrary angles and lengths.
def test_l1_segment_general():
    rng = np.random.default_rng(4)
    for K in (3, 8, 16):
        for _ in range(5):
            th = np.sort(rng.uniform(0, 2 * math.pi, K))
            while np.max(np.diff(np.r_[th, th[0] + 2 * math.pi])) >= math.pi:
                th = np.sort(rng.uniform(0, 2 * math.pi, K))
            s = rng.uniform(0.2, 2.0, K)
            e = np.stack([s * np.cos(th), s * np.sin(th)], -1)
            k = rng.integers(0, K, 200)
            lam, mu = rng.uniform(0.01, 2.0, (2, 200))
            p = lam[:, None] * e[k] + mu[:, None] * e[(k + 1) % K]
            a = _alpha(p[:, 0], p[:, 1], s, th, 1.0, 0.0, 1.0)
            np.testing.assert_allclose(a, np.exp(-0.5 * (lam + mu) ** 2), rtol=1e-10)


# ---- Sec. 4.1: inside a sector at phi = delta/3 the cosine weight is cos(pi/3) = 1/2, so
# 1/sbar^2 = 3/(4 s_k^2) + 1/(4 s_{k+1}^2); on a basis direction it is 1/s_k^2.
def test_l2_interpolation_points():
    rng = np.random.default_rng(5)
    K = 8
    th = np.sort(rng.uniform(0, 2 * math.pi, K))
    while np.max(np.diff(np.r_[th, th[0] + 2 * math.pi])) >= math.pi:
        th = np.sort(rng.uniform(0, 2 * math.pi, K))
    s = rng.uniform(0.2, 2.0, K)
    for k in range(K):
        t0 = th[k]
        t1 = th[k + 1] if k + 1 < K else th[0] + 2 * math.pi
        ang = t0 + (t1 - t0) / 3
        r = rng.uniform(0.1, 2.0)
        a = _alpha([r * math.cos(ang)], [r * math.sin(ang)], s, th, 0.0, 0.0, 1.0)[0]
        w = 3 / (4 * s[k] ** 2) + 1 / (4 * s[(k + 1) % K] ** 2)
        assert a == pytest.approx(math.exp(-0.5 * r * r * w), rel=1e-12)
        a = _alpha([r * math.cos(t0)], [r * math.sin(t0)], s, th, 0.0, 0.0, 1.0)[0]
        assert a == pytest.approx(math.exp(-0.5 * r * r / s[k] ** 2), rel=1e-10)


# ---- Sec. 4.3 sharpening: continuity, fixed points, symmetry, slopes, identity at tau = 0
@pytest.mark.parametrize("tau", [-0.9, -0.1, 0.0, 0.3, 0.5, 0.99])
def test_p4_psi_identities(tau):
    t = torch.tensor(tau, dtype=F64)
    for gval, want in ((0.0, 0.0), (0.5, 0.5), (1.0, 1.0)):
        assert float(O.psi(torch.tensor(gval, dtype=F64), t)) == pytest.approx(want, abs=1e-14)
    g = torch.linspace(0, 1, 20001, dtype=F64)
    y = O.psi(g, t)
    assert torch.all(torch.diff(y) > 0)                                  # strictly increasing
    np.testing.assert_allclose((1 - O.psi(1 - g, t)).numpy(), y.numpy(), atol=1e-14)  # point symmetry
    for b in ((1 + tau) / 4, (3 - tau) / 4):                               # continuity at breakpoints
        lo = O.psi(torch.tensor(b - 1e-12, dtype=F64), t)
        hi = O.psi(torch.tensor(b, dtype=F64), t)
        steep = max((1 + tau) / (1 - tau), (1 - tau) / (1 + tau))
        assert abs(float(hi - lo)) <= 1.01e-12 * steep + 1e-15
    slope_in = float((O.psi(torch.tensor(0.01, dtype=F64), t)) / 0.01)
    assert slope_in == pytest.approx((1 - tau) / (1 + tau), rel=1e-12)
    eps = (1 - abs(tau)) / 10            # inside the middle piece [(1+tau)/4, (3-tau)/4)
    mid = torch.tensor([0.5 - eps, 0.5 + eps], dtype=F64)
    ym = O.psi(mid, t)
    assert float((ym[1] - ym[0]) / (2 * eps)) == pytest.approx((1 + tau) / (1 - tau), rel=1e-9)
    yy = torch.linspace(0, 1, 1001, dtype=F64)
    np.testing.assert_allclose(O.psi(O.psi_inv(yy, t), t).numpy(), yy.numpy(), atol=1e-13)
    if tau == 0.0:
        np.testing.assert_allclose(y.numpy(), g.numpy(), atol=0)


# ---- Sec. 4.4 (calibrated length, corrected): on the level set E = c^2 the opacity equals alpha_min
def test_calibrated_radius_level():
    rng = np.random.default_rng(6)
    amin = 1.0 / 255.0
    o = _t(rng.uniform(0.01, 0.99, 1000))
    tau = _t(rng.uniform(-0.5, 0.99, 1000))
    c = O.calibrated_radius(o, tau, amin)
    a = o * O.psi(torch.exp(-0.5 * c * c), tau)
    np.testing.assert_allclose(a.numpy(), amin, rtol=1e-10)


# ---- Real SH against scipy's complex harmonics (Y_lm real = sqrt2 (-1)^m Re/Im of Y_l^|m|)
def test_real_sh_matches_scipy():
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(7)
    d = rng.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    polar = np.arccos(np.clip(d[:, 2], -1, 1))
    azim = np.arctan2(d[:, 1], d[:, 0])
    Y = O.real_sh(3, _t(d)).numpy()
    for l in range(4):
        for m in range(-l, l + 1):
            if m == 0:
                ref = sph_harm_y(l, 0, polar, azim).real
            elif m > 0:
                ref = math.sqrt(2) * (-1) ** m * sph_harm_y(l, m, polar, azim).real
            else:
                ref = math.sqrt(2) * (-1) ** m * sph_harm_y(l, -m, polar, azim).imag
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-12, err_msg=f"l={l} m={m}")


# ---- Sec. 3.3 ray-plane intersection: (u, v) and r_t against a 3x3 linear solve
#      r_o + t r_d = mu + u t_u + v t_v
def test_hit_against_linear_solve():
    rng = np.random.default_rng(8)
    W = H = 32
    fx, fy, cx, cy = intrinsics_hfov(W, H, 60.0)
    Rw, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Rw = (Rw * np.sign(np.linalg.det(Rw))).astype(np.float32)
    eye = np.array([0.3, -0.2, -5.0])
    t = (-(Rw.astype(np.float64) @ eye)).astype(np.float32)
    cam = O.Cam.from_camera(Camera(W, H, fx, fy, cx, cy, Rw, t))
    n = 40
    mu = (eye + (Rw.astype(np.float64).T @ np.array([0, 0, 5.0])) + rng.normal(0, 0.5, (n, 3))).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    P = O.Prims(_t(mu), _t(q), _t(np.full((n, 4), 0.5)), _t(np.tile([0, 1.5, 3, 4.5], (n, 1))),
                _t(np.zeros(n)), _t(np.zeros(n)), _t(np.full(n, 0.9)), _t(np.ones((n, 3))), -1)
    px = torch.as_tensor(rng.integers(0, W, n))
    py = torch.as_tensor(rng.integers(0, H, n))
    res = O.eval_pairs(P, cam, O.Opts(lowpass_sl=0.0), px, py, P.color)
    Rq = O.quat_to_rotmat(_t(q)).numpy()
    # camera model X_c = R X_w + t: the centre solves R r_o + t = 0 and a pixel's ray direction solves
    # R r_d = K^-1 (px, py, 1) (R is float32, so R^T is not exactly its inverse)
    Rc = cam.R.numpy()
    ro = np.linalg.solve(Rc, -cam.t.numpy())
    for i in range(n):
        dcam = np.array([(px[i].item() + 0.5 - cam.cx) / cam.fx, (py[i].item() + 0.5 - cam.cy) / cam.fy, 1.0])
        rd = np.linalg.solve(Rc, dcam)
        rd /= np.linalg.norm(rd)
        A = np.stack([rd, -Rq[i][:, 0], -Rq[i][:, 1]], 1)
        tt, uu, vv = np.linalg.solve(A, mu[i].astype(np.float64) - ro)
        assert res["u"][i].item() == pytest.approx(uu, rel=1e-9, abs=1e-12)
        assert res["v"][i].item() == pytest.approx(vv, rel=1e-9, abs=1e-12)
        assert res["rt"][i].item() == pytest.approx(tt, rel=1e-9)


# ---- P5 analytic footprint: one fronto-parallel Gaussian-case DRK at depth d in front of a
# camera at the origin; u = d (x + 0.5 - cx)/fx, v = d (y + 0.5 - cy)/fy exactly, and the image is
# alpha*c + (1 - alpha)*bg with alpha from Eq. (3) (clamped and cut as the 3D-GS cutoffs say).
def test_p5_single_primitive_footprint():
    W, H = 48, 40
    fx, fy, cx, cy = intrinsics_hfov(W, H, 60.0)
    d, su, sv, o = 3.0, 0.4, 0.25, 0.8
    col = np.array([0.9, 0.4, 0.1], np.float32)
    bg = np.array([0.1, 0.2, 0.3], np.float32)
    sc = Scene(np.array([[0.0], [0.0], [d]], np.float32), np.array([[1.0], [0], [0], [0]], np.float32),
               np.array([[su], [sv], [su], [sv]], np.float32),
               np.array([[0.0], [math.pi / 2], [math.pi], [1.5 * math.pi]], np.float32),
               np.zeros(1, np.float32), np.zeros(1, np.float32), np.array([o], np.float32), col[:, None], -1)
    cam = Camera(W, H, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.zeros(3, np.float32), bg)
    opts = O.Opts(lowpass_sl=0.0)
    r = O.render_image(sc, cam, opts)
    yy, xx = np.mgrid[0:H, 0:W]
    u = d * (xx + 0.5 - float(cx)) / float(fx)
    v = d * (yy + 0.5 - float(cy)) / float(fy)
    su32, sv32, o32 = (float(np.float32(x)) for x in (su, sv, o))
    a = o32 * np.exp(-0.5 * (u ** 2 / su32 ** 2 + v ** 2 / sv32 ** 2))
    a = np.minimum(a, opts.alpha_max)
    a = np.where(a >= opts.alpha_min, a, 0.0).ravel()
    ref = a[:, None] * col.astype(np.float64)[None] + (1 - a)[:, None] * bg.astype(np.float64)[None]
    np.testing.assert_allclose(r.rgb, ref, atol=1e-12)
    np.testing.assert_allclose(r.T, 1 - a, atol=1e-12)


# ---- Eq. (1): two primitives in front of each other composite in closed form
def test_two_layer_composite_closed_form():
    C, T, n, w = O.composite([0.3, 0.6], [[1, 0, 0], [0, 1, 0]], [0, 0, 1], 1e-4)
    assert C == pytest.approx([0.3, 0.7 * 0.6, 0.7 * 0.4])
    assert T == pytest.approx(0.28) and n == 2
    # stop rule: T * (1 - a) < T_min ends the pixel without adding that contribution
    C, T, n, w = O.composite([0.99, 0.99, 0.99], [[1, 1, 1]] * 3, [0, 0, 0], 2e-4)
    assert n == 1 and T == pytest.approx(0.01) and C == pytest.approx([0.99] * 3)
    C, T, n, w = O.composite([0.99, 0.99, 0.99], [[1, 1, 1]] * 3, [0, 0, 0], 5e-5)
    assert n == 2 and T == pytest.approx(1e-4)


# ---- P6 telescoping: sum_i T_i alpha_i + T_final = 1 on the full 64x64 workload
def test_p6_weights_telescope_c1():
    scene, cam = config_c1()
    r = O.render_image(scene, cam, O.Opts())
    w = np.array([sum(x) for x in r.weights])
    np.testing.assert_allclose(w + r.T, 1.0, atol=1e-12)
    assert r.n_contrib.max() > 3           # the workload really overlaps


# ---- P7 cache semantics (Algorithm 1) against a bounded heap, plus its special cases
def _heap_emit(seq, L):
    h, out = [], []
    for i, (rt, j) in enumerate(seq):
        if len(h) >= L:
            out.append(heapq.heappop(h)[2:])
        heapq.heappush(h, (rt, i, rt, j))
    while h:
        out.append(heapq.heappop(h)[2:])
    return [tuple(x) for x in out]


def test_p7_cache_semantics():
    rng = np.random.default_rng(9)
    for _ in range(300):
        n = int(rng.integers(0, 30))
        L = int(rng.integers(1, 12))
        rts = rng.integers(0, 10, n).astype(float)        # many ties
        seq = [(float(rts[i]), i) for i in range(n)]
        assert O.cache_emit(seq, L) == _heap_emit(seq, L)
        assert O.cache_emit(seq, 1) == seq                                  # L = 1: arrival order
        assert O.cache_emit(seq, max(n, 1)) == sorted(seq, key=lambda x: (x[0], x[1]))  # L >= n: exact
    s = [(float(i), i) for i in range(20)]
    assert O.cache_emit(s, 8) == s                                          # sorted input unchanged
    r = [(float(8 - i), i) for i in range(8)]
    assert O.cache_emit(r, 8) == sorted(r)                                  # reversed input, n <= L


# ---- Two Gaussian-reduced DRKs on planes that cross along the optical axis (Sec. 4.1 reduction,
# Eq. 1, Sec. 4.4 Cache Sorting): their centres coincide, so the centre-depth pre-sort is the index
# order on every pixel, while the hit depths swap sides at the crossing.  Every expected value is
# elementary geometry written out here: ray-plane hit, in-plane distance, o exp(-r^2 / 2s^2), and the
# two-layer blend in hit-depth order (index order for a cache of one slot).
def test_crossing_planes_order_by_hit_depth():
    W, H, s, phi = 48, 32, 3.0, math.radians(30.0)
    o = (0.6, 0.5)
    col = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]], np.float32)    # A red, B green
    bg = np.array([0.0, 0.0, 1.0])
    K = 8
    q = np.array([[math.cos(phi / 2), math.cos(-phi / 2)], [0.0, 0.0],
                  [math.sin(phi / 2), math.sin(-phi / 2)], [0.0, 0.0]], np.float32)
    theta = np.tile((np.arange(K) * 2 * math.pi / K)[:, None], (1, 2)).astype(np.float32)
    sc = Scene(np.array([[0.0, 0.0], [0.0, 0.0], [4.0, 4.0]], np.float32), q, np.full((K, 2), s, np.float32), theta,
               np.zeros(2, np.float32), np.zeros(2, np.float32), np.array(o, np.float32), col, -1)
    fx, fy, cx, cy = intrinsics_hfov(W, H, 60.0)
    cam = Camera(W, H, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.zeros(3, np.float32), bg.astype(np.float32))
    # expected, from the float32 inputs in float64
    yy, xx = np.mgrid[0:H, 0:W]
    ray = np.stack([(xx.ravel() + 0.5 - float(cx)) / float(fx), (yy.ravel() + 0.5 - float(cy)) / float(fy),
                    np.ones(W * H)], 1)
    p0 = np.array([0.0, 0.0, 4.0])
    Z, alpha = [], []
    for j in range(2):
        w, y = float(q[0, j]), float(q[2, j])
        nrm = np.array([2 * w * y, 0.0, 1 - 2 * y * y]) / (w * w + y * y)   # third column of R(q)
        t = (nrm @ p0) / (ray @ nrm)
        hit = ray * t[:, None]
        r2 = ((hit - p0) ** 2).sum(1)
        Z.append(t)
        alpha.append(float(np.float32(o[j])) * np.exp(-r2 / (2 * float(np.float32(s)) ** 2)))
    Z, alpha = np.array(Z), np.array(alpha)

    def blend(first):
        f, b = first, 1 - first
        af, ab = alpha[f, np.arange(W * H)], alpha[b, np.arange(W * H)]
        return (af[:, None] * col.T[f] + ((1 - af) * ab)[:, None] * col.T[b]
                + ((1 - af) * (1 - ab))[:, None] * bg)

    by_depth = blend((Z[1] < Z[0]).astype(int))
    by_index = blend(np.zeros(W * H, int))
    assert (Z[0] < Z[1]).any() and (Z[1] < Z[0]).any()
    assert np.abs(by_depth - by_index).max() > 0.05
    for L, want in ((O.EXACT, by_depth), (8, by_depth), (2, by_depth), (1, by_index)):
        r = O.render_image(sc, cam, O.Opts(cache_len=L, lowpass_sl=0.0))
        assert not r.knife.any()
        np.testing.assert_allclose(r.rgb, want, atol=1e-7, err_msg=f"cache_len {L}")


# ---- The near plane cuts hits, not only centres: one Gaussian-reduced DRK on a steep plane whose
# centre lies just beyond the near plane.  Where the ray meets the plane at or before the near plane
# the pixel keeps the background; elsewhere it is o exp(-r^2 / 2s^2) over the background, from the
# ray-plane hit written out here.
def test_near_plane_cuts_hits_of_a_tilted_plane():
    W, H, s, phi, near, o = 40, 24, 2.0, math.radians(60.0), 0.9, 0.8
    K = 8
    q = np.array([[math.cos(phi / 2)], [0.0], [math.sin(phi / 2)], [0.0]], np.float32)
    theta = (np.arange(K) * 2 * math.pi / K)[:, None].astype(np.float32)
    sc = Scene(np.array([[0.0], [0.0], [1.0]], np.float32), q, np.full((K, 1), s, np.float32), theta,
               np.zeros(1, np.float32), np.zeros(1, np.float32), np.array([o], np.float32),
               np.array([[1.0], [1.0], [0.0]], np.float32), -1)
    fx, fy, cx, cy = intrinsics_hfov(W, H, 90.0)
    bg = np.array([0.0, 0.0, 1.0])
    cam = Camera(W, H, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.zeros(3, np.float32), bg.astype(np.float32))
    yy, xx = np.mgrid[0:H, 0:W]
    ray = np.stack([(xx.ravel() + 0.5 - float(cx)) / float(fx), (yy.ravel() + 0.5 - float(cy)) / float(fy),
                    np.ones(W * H)], 1)
    w, y = float(q[0, 0]), float(q[2, 0])
    nrm = np.array([2 * w * y, 0.0, 1 - 2 * y * y]) / (w * w + y * y)
    p0 = np.array([0.0, 0.0, 1.0])
    den = ray @ nrm
    Z = np.where(den > 0, (nrm @ p0) / np.where(den > 0, den, 1.0), -1.0)   # hit depth (ray z = 1)
    r2 = ((ray * Z[:, None] - p0) ** 2).sum(1)
    a = np.where(Z > near, float(np.float32(o)) * np.exp(-r2 / (2 * s * s)), 0.0)
    want = a[:, None] * np.array([1.0, 1.0, 0.0]) + (1 - a)[:, None] * bg
    cut = Z <= near
    assert cut.sum() > W * H // 10 and (~cut).sum() > W * H // 10
    r = O.render_image(sc, cam, O.Opts(near=near, lowpass_sl=0.0))
    ok = ~r.knife
    assert ok.sum() >= W * H - 2
    np.testing.assert_allclose(r.rgb[ok], want[ok], atol=1e-7)
    np.testing.assert_array_equal(r.n_emit[cut & ok], 0)


# ---- The alpha clamp and the alpha cutoff on one opaque fronto-parallel Gaussian-reduced DRK:
# alpha = min(exp(-r^2 / 2s^2), alpha_max) where that is at least alpha_min, else nothing.
def test_alpha_clamp_and_cutoff_of_one_opaque_drk():
    W = H = 49                      # odd: one pixel centre on the axis, where alpha is clamped
    s, depth, K = 0.3, 3.0, 8
    sc = Scene(np.array([[0.0], [0.0], [depth]], np.float32), np.array([[1.0], [0.0], [0.0], [0.0]], np.float32),
               np.full((K, 1), s, np.float32), (np.arange(K) * 2 * math.pi / K)[:, None].astype(np.float32),
               np.zeros(1, np.float32), np.zeros(1, np.float32), np.ones(1, np.float32),
               np.array([[0.2], [0.9], [0.4]], np.float32), -1)
    fx, fy, cx, cy = intrinsics_hfov(W, H, 60.0)
    bg = np.array([0.5, 0.0, 0.5])
    cam = Camera(W, H, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.zeros(3, np.float32), bg.astype(np.float32))
    yy, xx = np.mgrid[0:H, 0:W]
    u = (xx.ravel() + 0.5 - float(cx)) / float(fx) * depth
    v = (yy.ravel() + 0.5 - float(cy)) / float(fy) * depth
    g = np.exp(-(u * u + v * v) / (2 * float(np.float32(s)) ** 2))
    opts = O.Opts(lowpass_sl=0.0)
    amax, amin = float(np.float32(opts.alpha_max)), float(np.float32(opts.alpha_min))
    a = np.where(g >= amin, np.minimum(g, amax), 0.0)
    want = a[:, None] * np.array([0.2, 0.9, 0.4], np.float32).astype(np.float64) + (1 - a)[:, None] * bg
    assert (g > amax).sum() >= 1 and (g < amin).sum() > W * H // 4
    r = O.render_image(sc, cam, opts.f32())
    ok = ~r.knife
    assert ok[np.argmax(g)] and ok.sum() >= W * H - 4
    np.testing.assert_allclose(r.rgb[ok], want[ok], atol=1e-7)
    np.testing.assert_array_equal(r.n_emit[ok], (a[ok] > 0).astype(int))


# ---- View-dependent colour in the render (Sec. 3.1, SH as in 3D-GS): degree-1 SH evaluated at the
# direction from the camera centre to the DRK's centre, plus 0.5, clamped at 0, and the same colour
# on every pixel of that DRK.  The basis is written out: Y_0 = 1/(2 sqrt(pi)), (Y_1, Y_2, Y_3) =
# sqrt(3/(4 pi)) (y, z, x).
def test_sh_colour_of_an_off_axis_drk():
    W = H = 33
    mu = np.array([0.6, -0.4, 3.0])
    campos = np.array([0.2, 0.3, -1.0])
    K = 8
    coef = np.array([[0.1, -2.5, 0.3],      # l = 0, channels r g b
                     [0.5, 0.2, -0.6],      # Y_1 ~ y
                     [-0.3, 0.4, 0.1],      # Y_2 ~ z
                     [0.7, -0.2, 0.9]])     # Y_3 ~ x
    color = coef.reshape(12, 1).astype(np.float32)     # row 3 * coefficient + channel
    sc = Scene(mu[:, None].astype(np.float32), np.array([[1.0], [0.0], [0.0], [0.0]], np.float32),
               np.full((K, 1), 0.4, np.float32), (np.arange(K) * 2 * math.pi / K)[:, None].astype(np.float32),
               np.zeros(1, np.float32), np.zeros(1, np.float32), np.full(1, 0.9, np.float32), color, 1)
    fx, fy, cx, cy = intrinsics_hfov(W, H, 50.0)
    R = np.eye(3, dtype=np.float32)
    t = (-campos).astype(np.float32)
    cam = Camera(W, H, fx, fy, cx, cy, R, t, np.zeros(3, np.float32))
    d = mu.astype(np.float32).astype(np.float64) - campos.astype(np.float32).astype(np.float64)
    x, y, z = d / np.linalg.norm(d)
    Y = np.array([0.5 / math.sqrt(math.pi)] + [math.sqrt(3 / (4 * math.pi)) * c for c in (y, z, x)])
    rgb = np.maximum(Y @ coef.astype(np.float32).astype(np.float64) + 0.5, 0.0)
    assert rgb.min() == 0.0 and rgb.max() > 0.5                # one channel is clamped
    r = O.render_image(sc, cam, O.Opts(lowpass_sl=0.0))
    T = r.T
    hit = (r.n_emit == 1) & ~r.knife
    assert hit.sum() > 20
    # one layer over a black background: colour = (1 - T) * rgb
    np.testing.assert_allclose(r.rgb[hit], (1 - T[hit])[:, None] * rgb[None, :], atol=1e-9)


# ---- The transmittance stop in the render (Eq. 1 with the T_min rule): five fronto-parallel
# Gaussian-reduced DRKs stacked on the optical axis, each of opacity 0.92.  On the axis pixel every
# layer has alpha 0.92, so T runs 0.08, 0.0064, 5.12e-4, and the fourth layer (4.1e-5 < 1e-4) stops
# the pixel unadded: three layers composite and the background enters with T = 0.08^3.
def test_transmittance_stop_on_stacked_layers():
    W = H = 9
    K, n, s, o = 8, 5, 0.5, 0.92
    depths = 3.0 + 0.25 * np.arange(n)
    cols = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [0, 1, 1]], np.float32)
    sc = Scene(np.stack([np.zeros(n), np.zeros(n), depths]).astype(np.float32),
               np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)), np.full((K, n), s, np.float32),
               np.tile((np.arange(K) * 2 * math.pi / K)[:, None], (1, n)).astype(np.float32),
               np.zeros(n, np.float32), np.zeros(n, np.float32), np.full(n, o, np.float32), cols.T.copy(), -1)
    fx, fy, cx, cy = intrinsics_hfov(W, H, 30.0)
    bg = np.array([0.3, 0.3, 0.3])
    cam = Camera(W, H, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.zeros(3, np.float32), bg.astype(np.float32))
    r = O.render_image(sc, cam, O.Opts(lowpass_sl=0.0))
    c = (H // 2) * W + W // 2
    a = float(np.float32(o))
    Ts = [1.0, 1 - a, (1 - a) ** 2, (1 - a) ** 3]
    want = sum(Ts[i] * a * cols[i].astype(np.float64) for i in range(3)) + Ts[3] * bg
    assert Ts[3] * (1 - a) < 1e-4 <= Ts[3]
    assert not r.knife[c] and r.n_emit[c] == 3
    assert r.emitted[c] == [0, 1, 2]
    np.testing.assert_allclose(r.rgb[c], want, atol=1e-12)
    assert r.T[c] == pytest.approx(Ts[3], rel=1e-12)


# ---- P8: fronto-parallel scene (all normals along the optical axis): r_t order equals centre-depth
# order, so the 8-slot cache reproduces the exact per-pixel sort.
def test_p8_frontoparallel_cache_equals_exact():
    scene, cam = config_c1()
    sc = Scene(scene.mu.copy(), np.tile(np.array([[1.0], [0], [0], [0]], np.float32), (1, scene.n)),
               scene.scale, scene.theta, scene.eta, scene.tau, scene.opacity, scene.color, -1)
    a = O.render_image(sc, cam, O.Opts(cache_len=8))
    b = O.render_image(sc, cam, O.Opts(cache_len=O.EXACT))
    c = O.render_image(sc, cam, O.Opts(cache_len=1))
    np.testing.assert_allclose(a.rgb, b.rgb, atol=1e-13)
    np.testing.assert_allclose(c.rgb, b.rgb, atol=1e-13)


# ---- P9 culling is conservative: every sampled tangent-plane point with E <= c^2 lies inside
# the support polygon, and binning the pixels by the tile lists changes no pixel.
def _inside(poly, pts):
    x, y = pts[:, 0], pts[:, 1]
    inside = np.zeros(len(pts), bool)
    n = len(poly)
    for i in range(n):
        x0, y0 = poly[i]
        x1, y1 = poly[(i + 1) % n]
        cond = ((y0 > y) != (y1 > y))
        xint = x0 + (y - y0) * (x1 - x0) / np.where(y1 != y0, y1 - y0, 1)
        inside ^= cond & (x < xint)
    return inside


def test_p9_support_polygon_contains_support():
    rng = np.random.default_rng(10)
    scene, _ = config_c1()
    for j in range(60):
        s = scene.scale[:, j].astype(np.float64)
        th = scene.theta[:, j].astype(np.float64)
        o, tau, eta = float(scene.opacity[j]), float(scene.tau[j]), float(scene.eta[j])
        c = float(O.calibrated_radius(_t(o), _t(tau), 1 / 255))
        poly = O.support_polygon(s, th, c)
        R = c * s.max() * 1.05
        pts = rng.uniform(-R, R, (20000, 2))
        a = _alpha(pts[:, 0], pts[:, 1], s, th, eta, tau, o)
        supp = a >= 1 / 255
        assert supp.any()
        assert _inside(poly, pts[supp]).all(), j


def test_p9_binning_changes_no_pixel_c1():
    scene, cam = config_c1()
    opts = O.Opts()
    tiles, per, key = O.tile_lists(scene, cam, opts)
    members = {t: {j for _, j in v} for t, v in tiles.items()}
    a = O.render_image(scene, cam, opts)
    b = O.render_image(scene, cam, opts, tile_members=members)
    np.testing.assert_array_equal(a.rgb, b.rgb)
    np.testing.assert_array_equal(a.n_emit, b.n_emit)


def test_prefilter_is_lossless_c1():
    scene, cam = config_c1()
    a = O.render_image(scene, cam, O.Opts())
    b = O.render_image(scene, cam, O.Opts(), prefilter=False)
    np.testing.assert_array_equal(a.rgb, b.rgb)


# ---- The paper's printed endpoint polygon (Sec. 4.4) is not conservative: it misses support.
def test_paper_polygon_misses_support():
    rng = np.random.default_rng(11)
    scene, _ = config_c1()
    missed = 0
    for j in range(30):
        s = scene.scale[:, j].astype(np.float64)
        th = scene.theta[:, j].astype(np.float64)
        o, tau, eta = float(scene.opacity[j]), float(scene.tau[j]), float(scene.eta[j])
        poly = O.paper_polygon(s, th, o, tau)
        R = 6 * s.max()
        pts = rng.uniform(-R, R, (20000, 2))
        supp = _alpha(pts[:, 0], pts[:, 1], s, th, eta, tau, o) >= 1 / 255
        missed += int((~_inside(poly, pts[supp])).sum())
    assert missed > 0


# ---- P10 gradients: Eq. (3) closed-form derivatives in the Gaussian case, and central finite
# differences of the full render for a small scene.
def test_p10_gaussian_scale_gradient_closed_form():
    rng = np.random.default_rng(12)
    su, sv, o = 0.6, 0.3, 0.7
    u, v = rng.normal(0, 0.5, (2, 50))
    s = torch.tensor([su, sv, su, sv], dtype=F64, requires_grad=True)
    th = torch.tensor([0, math.pi / 2, math.pi, 1.5 * math.pi], dtype=F64)
    L = len(u)
    a = O.drk_alpha_uv(_t(u), _t(v), s.expand(L, 4), th.expand(L, 4), torch.zeros(L, dtype=F64),
                       torch.zeros(L, dtype=F64), torch.full((L,), o, dtype=F64))
    a.sum().backward()
    g = o * np.exp(-0.5 * (u ** 2 / su ** 2 + v ** 2 / sv ** 2))
    dsu = (g * u ** 2 / su ** 3).sum()
    dsv = (g * v ** 2 / sv ** 3).sum()
    gs = s.grad.numpy()
    assert gs[0] + gs[2] == pytest.approx(dsu, rel=1e-10)
    assert gs[1] + gs[3] == pytest.approx(dsv, rel=1e-10)


def _small_scene(seed, n=12, sh=False):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-0.5, 0.5, (3, n)).astype(np.float32)
    q = rng.normal(size=(4, n)).astype(np.float32)
    K = 8
    from drk_synth import draw_angles
    th = draw_angles(rng, K, n)
    s = np.exp(rng.uniform(math.log(0.15), math.log(0.6), (K, n))).astype(np.float32)
    eta = rng.uniform(0, 1, n).astype(np.float32)
    tau = rng.uniform(0, 0.9, n).astype(np.float32)
    o = rng.uniform(0.3, 0.95, n).astype(np.float32)
    if sh:
        col = rng.normal(0, 0.1, (48, n)).astype(np.float32)
        col[:3] = rng.uniform(0, 1, (3, n))
        return Scene(mu, q, s, th, eta, tau, o, col, 3)
    return Scene(mu, q, s, th, eta, tau, o, rng.uniform(0, 1, (3, n)).astype(np.float32), -1)


def test_p10_render_gradient_finite_differences():
    sc = _small_scene(13, sh=True)
    W = H = 16
    fx, fy, cx, cy = intrinsics_hfov(W, H, 60.0)
    cam = Camera(W, H, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.array([0, 0, 2.5], np.float32),
                 np.array([0.2, 0.1, 0.0], np.float32))
    yy, xx = np.mgrid[0:H, 0:W]
    px, py = xx.ravel(), yy.ravel()
    rng = np.random.default_rng(14)
    target = rng.uniform(0, 1, (len(px), 3))
    opts = O.Opts()
    loss, grads, rgb, fwd = O.render_loss_grad(sc, cam, opts, px, py, target)
    assert loss > 0
    # loss as a function of float64 parameters, emission order / decisions frozen as in the forward
    base = O.Prims.from_scene(sc)

    def loss_of(P):
        with torch.no_grad():
            colors = O.prim_colors(P, O.Cam.from_camera(cam))
            out = np.zeros((len(px), 3))
            for p, em in enumerate(fwd.emitted):
                T = 1.0
                for j in em:
                    r = O.eval_pairs(P.index(torch.tensor([j])), O.Cam.from_camera(cam), opts,
                                     torch.tensor([px[p]]), torch.tensor([py[p]]), colors[[j]])
                    a = float(r["alpha"][0])
                    out[p] += T * a * colors[j].numpy()
                    T *= (1 - a)
                out[p] += T * cam.bg.astype(np.float64)
            return ((out - target) ** 2).sum()

    assert loss_of(base) == pytest.approx(loss, rel=1e-12)
    checked = 0
    for name, shape_idx in (("mu", (0, 1)), ("q", (1, 2)), ("s", (2, 3)), ("theta", (3, 4)), ("eta", (4,)),
                            ("tau", (5,)), ("o", (6,)), ("color", (7, 0, 1))):
        g = grads[name]
        flat_idx = int(torch.argmax(g.abs().reshape(-1)))
        P1 = O.Prims.from_scene(sc)
        P2 = O.Prims.from_scene(sc)
        x = getattr(base, name).reshape(-1)[flat_idx].item()
        h = 1e-6 * max(1.0, abs(x))
        getattr(P1, name).reshape(-1)[flat_idx] += h
        getattr(P2, name).reshape(-1)[flat_idx] -= h
        fd = (loss_of(P1) - loss_of(P2)) / (2 * h)
        assert g.reshape(-1)[flat_idx].item() == pytest.approx(fd, rel=1e-5, abs=1e-8), name
        checked += 1
    assert checked == 8


# ---- P11: 74 float32 values per DRK (mu 3, q 4, s 8, theta 8, eta, tau, o, SH3 48) reproduce the
# model sizes of Table 2 (counts printed to three significant figures).
def test_p11_record_size_matches_table2():
    path = os.path.join(os.path.dirname(__file__), "golden", "table2_model_sizes.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    floats = 3 + 4 + 8 + 8 + 1 + 1 + 1 + 48
    assert floats == 74
    for name, count_k, mb in rows:
        est = float(count_k) * 1e3 * floats * 4 / 1e6
        # counts carry 2-3 significant figures; 1 MB = 1e6 bytes
        assert abs(est - float(mb)) / float(mb) < 0.012, (name, est, mb)
    # the same accounting for 3D-GS (59 floats: mu 3, q 4, s 3, o, SH3 48): 336K -> 79.7 MB in Table 2
    assert abs(336e3 * 59 * 4 / 1e6 - 79.7) / 79.7 < 0.012


# ---- P9 (adversarial): thin sectors, extreme length ratios, K in {3, 8, 16}, eta in {0, 1, U}, sharp
# and soft tau; points sampled densely near the support boundary must lie inside the polygon, and the
# polygon stays within the disc of radius sqrt(2) c max_k s_k used by the frustum cull.
def test_p9_support_polygon_adversarial():
    rng = np.random.default_rng(110)
    from drk_synth import draw_angles
    for trial in range(60):
        K = (3, 8, 16)[trial % 3]
        th = draw_angles(rng, K, 1)[:, 0].astype(np.float64)
        s = np.exp(rng.uniform(math.log(0.005), math.log(0.5), K))
        eta = (0.0, 1.0, float(rng.uniform()))[trial % 3]
        tau = float(rng.uniform(-0.9, 0.99))
        o = float(rng.uniform(0.02, 1.0))
        c = float(O.calibrated_radius(_t(o), _t(tau), 1 / 255))
        poly = O.support_polygon(s, th, c)
        assert np.hypot(poly[:, 0], poly[:, 1]).max() <= math.sqrt(2) * c * s.max() * (1 + 1e-12)
        ang = rng.uniform(0, 2 * math.pi, 40000)
        rad = c * s.max() * rng.uniform(0, 1, 40000) ** 0.5
        pts = np.stack([rad * np.cos(ang), rad * np.sin(ang)], -1)
        supp = _alpha(pts[:, 0], pts[:, 1], s, th, eta, tau, o) >= 1 / 255
        assert _inside(poly, pts[supp]).all(), trial


# ---- Pre-sort key variants and sorting-accuracy measures (supplement, cache-sorting evaluation)
def test_sort_metrics_hand_examples():
    m = O.sort_metrics([[1.0, 2.0, 3.0]])
    assert (m["accuracy"], m["kendall_tau"], m["mae"]) == (1.0, 1.0, 0.0)
    m = O.sort_metrics([[3.0, 2.0, 1.0]])
    assert m["accuracy"] == pytest.approx(1 / 3) and m["kendall_tau"] == -1.0 and m["mae"] == pytest.approx(4 / 3)
    # ties count as neither concordant nor discordant; equal depths at a position count as correct
    m = O.sort_metrics([[2.0, 1.0, 3.0, 3.0]])
    assert m["accuracy"] == 0.5 and m["kendall_tau"] == 0.5 and m["mae"] == 0.5
    # pooled over pixels: accuracy and MAE per element, tau per pixel; single-element pixels carry no tau
    m = O.sort_metrics([[1.0, 2.0], [2.0, 1.0], [5.0]], cap=None)
    assert m["accuracy"] == pytest.approx(3 / 5) and m["kendall_tau"] == 0.0 and m["pixels"] == 2
    assert O.sort_metrics([[3.0, 2.0, 1.0, 0.0]], cap=2)["kendall_tau"] == -1.0


def test_kendall_tau_matches_scipy():
    scipy_stats = pytest.importorskip("scipy.stats")
    rng = np.random.default_rng(41)
    for m in (2, 3, 7, 40):
        for _ in range(5):
            z = rng.permutation(m).astype(np.float64) + rng.uniform(0, 0.5, m)
            ref = scipy_stats.kendalltau(np.arange(m), z).statistic
            assert O.sort_metrics([z])["kendall_tau"] == pytest.approx(ref, abs=1e-12)


def _tilted_scene(seed, n=40, K=8):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-0.6, 0.6, (3, n)).astype(np.float32)
    q = rng.normal(size=(4, n)).astype(np.float32)
    th = np.sort(rng.uniform(0, 2 * math.pi, (n, K)), 1)
    th[:, :] = (np.arange(K)[None, :] + rng.uniform(0.1, 0.9, (n, K))) * (2 * math.pi / K)
    s = np.exp(rng.uniform(math.log(0.1), math.log(0.6), (K, n))).astype(np.float32)
    return Scene(mu, q, s, th.T.astype(np.float32), rng.uniform(0, 1, n).astype(np.float32),
                 rng.uniform(0, 0.9, n).astype(np.float32), rng.uniform(0.3, 0.95, n).astype(np.float32),
                 rng.uniform(0, 1, (3, n)).astype(np.float32), -1)


def _cam_tilted(W=96, H=80):
    fx, fy, cx, cy = intrinsics_hfov(W, H, 60.0)
    a = 0.35
    R = np.array([[math.cos(a), 0, -math.sin(a)], [0, 1, 0], [math.sin(a), 0, math.cos(a)]], np.float32)
    return Camera(W, H, fx, fy, cx, cy, R, np.array([0.1, -0.05, 2.6], np.float32), np.zeros(3, np.float32))


def _depth_world(scene, cam, j, x, y):
    """View depth where the rays through pixel points (x, y) (arrays) meet DRK j's plane, from the
    world-space ray-plane intersection of Sec. 3.3 (independent of the camera-frame form the keys
    use)."""
    Rc = np.asarray(cam.R, np.float32).astype(np.float64)
    t = np.asarray(cam.t, np.float32).astype(np.float64)
    ro = -np.linalg.solve(Rc, t)
    f64 = lambda a: np.float64(np.float32(a))
    x, y = np.atleast_1d(np.asarray(x, np.float64)), np.atleast_1d(np.asarray(y, np.float64))
    dcam = np.stack([(x - f64(cam.cx)) / f64(cam.fx), (y - f64(cam.cy)) / f64(cam.fy), np.ones_like(x)])
    d = np.linalg.solve(Rc, dcam)                      # (3, P) world directions
    q = scene.q[:, j].astype(np.float64)
    n = O.quat_to_rotmat(torch.as_tensor(q))[:, 2].numpy()
    mu = scene.mu[:, j].astype(np.float64)
    rt = ((mu - ro) @ n) / (n @ d)
    return rt * (Rc[2] @ d)


def test_tile_keys_fronto_parallel_equal_centre_depth():
    """A DRK parallel to the image plane has one depth everywhere: both per-tile keys equal the
    centre-depth key."""
    sc = _tilted_scene(5)
    sc.q[:] = np.array([[1.0], [0.0], [0.0], [0.0]], np.float32)
    fx, fy, cx, cy = intrinsics_hfov(64, 48, 60.0)
    cam = Camera(64, 48, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.array([0, 0, 3.0], np.float32),
                 np.zeros(3, np.float32))
    centre = O.centre_depth_f32(sc.mu, cam)
    for mode in (O.KEY_CENTRIC, O.KEY_NEAREST):
        opts = O.Opts(key_mode=mode).f32()
        for j in range(sc.n):
            kp = O.key_plane(sc, cam, opts, j)
            for t in O.primitive_tiles(sc, cam, opts, j):
                k = np.uint32(O.tile_key(kp, cam, opts, t)).view(np.float32)
                assert abs(float(k) - float(centre[j])) <= 2e-7 * float(centre[j]), (mode, j, t)


def test_nearest_key_is_the_minimum_over_the_tile_brute_force():
    """The nearest key is the smallest plane depth over the kernel's part of the tile (checked on a
    33 x 33 grid of that rectangle with the world-space intersection), and the centric key is the
    depth at the rectangle's centre; both then held to the support's depth range."""
    sc, cam = _tilted_scene(6), _cam_tilted()
    checked = 0
    for mode in (O.KEY_CENTRIC, O.KEY_NEAREST):
        opts = O.Opts(key_mode=mode).f32()
        for j in range(sc.n):
            kp = O.key_plane(sc, cam, opts, j)
            for t in O.primitive_tiles(sc, cam, opts, j):
                xa, xb, ya, yb = O.key_rect(kp, cam, t)
                gx, gy = np.meshgrid(np.linspace(xa, xb, 33), np.linspace(ya, yb, 33))
                z = _depth_world(sc, cam, j, gx.ravel(), gy.ravel())
                if not (z > opts.near).all():
                    continue      # the plane turns away inside the rectangle: fallbacks apply
                ref = z.min() if mode == O.KEY_NEAREST else \
                    _depth_world(sc, cam, j, 0.5 * (xa + xb), 0.5 * (ya + yb))[0]
                ref = min(max(ref, kp.zlo), kp.zhi)
                assert O.tile_key_value(kp, cam, opts, t, mode) == pytest.approx(ref, rel=1e-9), (mode, j, t)
                checked += 1
    assert checked > 100


def test_nearest_key_never_after_centric_key():
    sc, cam = _tilted_scene(7), _cam_tilted()
    o1, o2 = O.Opts(key_mode=O.KEY_CENTRIC).f32(), O.Opts(key_mode=O.KEY_NEAREST).f32()
    n = 0
    for j in range(sc.n):
        kp = O.key_plane(sc, cam, o1, j)
        for t in O.primitive_tiles(sc, cam, o1, j):
            xa, xb, ya, yb = O.key_rect(kp, cam, t)
            if all(O.plane_depth(kp, cam, o1, x, y) is not None for x in (xa, xb) for y in (ya, yb)):
                assert O.tile_key_value(kp, cam, o2, t, O.KEY_NEAREST) <= O.tile_key_value(kp, cam, o1, t,
                                                                                         O.KEY_CENTRIC)
                n += 1
    assert n > 100


def test_support_depth_range_contains_polygon():
    """Every vertex of the support polygon lifted to the camera frame has a view depth within the
    support disc's range [zlo, zhi] (zlo before its clamp at the near plane)."""
    sc, cam = _tilted_scene(8), _cam_tilted()
    opts = O.Opts().f32()
    Rc = np.asarray(cam.R, np.float32).astype(np.float64)
    t = np.asarray(cam.t, np.float32).astype(np.float64)
    for j in range(sc.n):
        kp = O.key_plane(sc, cam, opts, j)
        o, tau = float(sc.opacity[j]), float(sc.tau[j])
        c = float(O.calibrated_radius(torch.tensor(o, dtype=F64), torch.tensor(tau, dtype=F64), opts.alpha_min))
        poly = O.support_polygon(sc.scale[:, j].astype(np.float64), sc.theta[:, j].astype(np.float64), c)
        R = O.quat_to_rotmat(torch.as_tensor(sc.q[:, j].astype(np.float64))).numpy()
        w = sc.mu[:, j].astype(np.float64)[None, :] + poly[:, :1] * R[:, 0] + poly[:, 1:] * R[:, 1]
        z = (w @ Rc.T + t)[:, 2]
        zr = kp.zhi - kp.zc
        assert z.max() <= kp.zhi + 1e-12 and z.min() >= kp.zc - zr - 1e-12


def test_per_tile_keys_change_order_not_images_of_separated_layers():
    """With well separated depth layers every pre-sort key gives the exact front-to-back order,
    so the three key modes give the same image as the exact sort."""
    rng = np.random.default_rng(9)
    n, K = 12, 8
    # one DRK per layer, tilted by about 0.1 rad: each spans at most +-0.09 in depth, 0.25 apart
    mu = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.3, 0.3, n), rng.permutation(n) * 0.25])
    q = np.tile(np.array([[1.0], [0.05], [0.0], [0.0]]), (1, n))
    th = (np.arange(K)[:, None] + 0.5) * (2 * math.pi / K) + np.zeros((1, n))
    sc = Scene(mu.astype(np.float32), q.astype(np.float32), np.full((K, n), 0.2, np.float32), th.astype(np.float32),
               np.full(n, 0.5, np.float32), np.zeros(n, np.float32), np.full(n, 0.6, np.float32),
               rng.uniform(0, 1, (3, n)).astype(np.float32), -1)
    fx, fy, cx, cy = intrinsics_hfov(32, 32, 60.0)
    cam = Camera(32, 32, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.array([0, 0, 3.0], np.float32),
                 np.zeros(3, np.float32))
    ref = O.render_image(sc, cam, O.Opts(cache_len=O.EXACT))
    for mode in (0, 1, 2):
        r = O.render_image(sc, cam, O.Opts(cache_len=1, key_mode=mode))
        np.testing.assert_allclose(r.rgb, ref.rgb, atol=1e-12)
        assert O.sort_metrics(r.emitted_z)["accuracy"] == 1.0


# ---- Mesh to DRK and the depth / normal channels (section "Converting Mesh to DRK" and supplement)
def _face_alpha(scene, j, pts_uv):
    s = scene.scale[:, j].astype(np.float64)
    th = scene.theta[:, j].astype(np.float64)
    return _alpha(pts_uv[:, 0], pts_uv[:, 1], s, th, float(scene.eta[j]), float(scene.tau[j]),
                  float(scene.opacity[j]))


def _to_uv(scene, j, P):
    R = O.quat_to_rotmat(torch.as_tensor(scene.q[:, j].astype(np.float64))).numpy()
    D = np.asarray(P, np.float64) - scene.mu[:, j].astype(np.float64)
    return np.stack([D @ R[:, 0], D @ R[:, 1]], -1)


@pytest.mark.parametrize("m,K", [(3, 3), (3, 5), (4, 4), (4, 8), (5, 8), (6, 16)])
def test_mesh_face_outline_is_the_half_opacity_contour(m, K):
    """Every vertex and every point of every edge of the face sits at alpha = o Psi(1/2) = o / 2; the
    centre is opaque and points 10% beyond the outline are transparent."""
    rng = np.random.default_rng(m * 100 + K)
    ang = np.sort(rng.uniform(0, 2 * math.pi, m))
    ang = 2 * math.pi * (np.arange(m) + rng.uniform(0.2, 0.8, m)) / m      # convex, gaps < pi
    rad = rng.uniform(0.5, 1.5, m)
    # a random plane in 3D
    R = O.quat_to_rotmat(torch.as_tensor(rng.normal(size=4))).numpy()
    c = rng.uniform(-1, 1, 3)
    P = c + (rad * np.cos(ang))[:, None] * R[:, 0] + (rad * np.sin(ang))[:, None] * R[:, 1]
    sc = O.mesh_to_drk(P, np.arange(m)[None, :], np.array([[0.2, 0.5, 0.9]]), K=K, tau=0.9, opacity=0.8)
    assert sc.opacity[0] == np.float32(0.8)
    uv = _to_uv(sc, 0, P)
    np.testing.assert_allclose(_face_alpha(sc, 0, uv), 0.4, atol=2e-5)
    t = np.linspace(0.05, 0.95, 7)
    edges = np.concatenate([uv[i] + t[:, None] * (uv[(i + 1) % m] - uv[i]) for i in range(m)])
    np.testing.assert_allclose(_face_alpha(sc, 0, edges), 0.4, atol=2e-5)
    assert _face_alpha(sc, 0, np.zeros((1, 2)))[0] == pytest.approx(0.8, abs=1e-6)
    # 10% outside: g < 1/2, Psi on its flat first piece; 10% inside: g > (3 - tau)/4, the flat last piece
    flat = (1 - 0.9) / (1 + 0.9)
    assert (_face_alpha(sc, 0, 1.1 * edges) <= 0.8 * flat * 0.5).all()
    assert (_face_alpha(sc, 0, 0.9 * edges) >= 0.8 * 2 * 0.9 / (1 + 0.9)).all()
    # the frame: the rotation of q has the face normal as its third column
    Rq = O.quat_to_rotmat(torch.as_tensor(sc.q[:, 0].astype(np.float64))).numpy()
    nrm = np.cross(P[1] - P[0], P[2] - P[1])
    np.testing.assert_allclose(Rq[:, 2], nrm / np.linalg.norm(nrm), atol=1e-6)


def test_mesh_rejects_degenerate_and_reversed_faces():
    V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [2, 0, 0], [0.6, 0.4, 0]], float)
    F = np.array([[0, 1, 2, 3], [0, 1, 4, -1], [0, 1, 5, 2], [0, 3, 2, 1], [0, 1, 2, -1]])
    sc = O.mesh_to_drk(V, F, np.ones((5, 3)), K=4)
    # square ok; collinear triangle degenerate; concave quad (gap >= pi at the reflex vertex is
    # impossible here, but the angles stop increasing); the square listed clockwise is a valid face
    # of the opposite normal; the triangle is padded to 4 bases
    assert sc.opacity[0] > 0 and sc.opacity[1] == 0 and sc.opacity[2] == 0 and sc.opacity[3] > 0 and sc.opacity[4] > 0
    R0 = O.quat_to_rotmat(torch.as_tensor(sc.q[:, 0].astype(np.float64))).numpy()
    R3 = O.quat_to_rotmat(torch.as_tensor(sc.q[:, 3].astype(np.float64))).numpy()
    np.testing.assert_allclose(R0[:, 2], -R3[:, 2], atol=1e-6)


def test_depth_and_normal_of_a_fronto_parallel_face():
    """A square face at depth 3 seen head-on: inside, the depth channel is alpha * 3 and the normal
    channel alpha * (0, 0, -1) (turned toward the camera), with alpha = min(o, 0.99); outside, both
    are zero."""
    z = 3.0
    V = np.array([[-0.5, -0.5, z], [0.5, -0.5, z], [0.5, 0.5, z], [-0.5, 0.5, z]])
    for F in (np.array([[0, 1, 2, 3]]), np.array([[3, 2, 1, 0]])):
        sc = O.mesh_to_drk(V, F, np.array([[1.0, 0.5, 0.25]]), K=4, tau=0.98, opacity=0.97)
        fx, fy, cx, cy = intrinsics_hfov(32, 32, 60.0)
        cam = Camera(32, 32, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.zeros(3, np.float32),
                     np.zeros(3, np.float32))
        r = O.render_image(sc, cam, O.Opts(lowpass_sl=0.0))
        # pixel (16, 16) is near the centre, pixel (0, 0) far outside
        c = 16 * 32 + 16
        a = r.T[c]
        assert r.depth[c] == pytest.approx((1 - a) * z, rel=1e-9)
        np.testing.assert_allclose(r.normal[c], [0, 0, -(1 - a)], atol=1e-9)
        assert 1 - a == pytest.approx(0.97, abs=1e-3)
        assert r.depth[0] == 0.0 and np.all(r.normal[0] == 0.0)


def test_depth_channel_is_the_weighted_sum_of_hit_depths():
    """depth = sum_i T_i alpha_i Z_i over the composited contributions, normal likewise with unit
    normals: the weights telescope with the transmittance."""
    scene, cam = config_c1()
    r = O.render_image(scene, cam, O.Opts())
    for p in np.nonzero(r.n_emit > 2)[0][:50]:
        assert r.depth[p] == pytest.approx(sum(w * z for w, z in zip(r.weights[p], r.emitted_z[p])), rel=1e-12)
        assert np.linalg.norm(r.normal[p]) <= sum(r.weights[p]) + 1e-12
        assert sum(r.weights[p]) + r.T[p] == pytest.approx(1.0, abs=1e-12)


# ---- Parametrization and Adam (supplement S4)
def _raw(n, K, seed, spread=3.0):
    rng = np.random.default_rng(seed)
    return {"mu": torch.as_tensor(rng.normal(size=(n, 3))), "q": torch.as_tensor(rng.normal(size=(n, 4))),
            "scale": torch.as_tensor(rng.normal(-2, 1, (n, K))), "theta": torch.as_tensor(rng.normal(0, spread, (n, K))),
            "eta": torch.as_tensor(rng.normal(size=n)), "tau": torch.as_tensor(rng.normal(size=n)),
            "opacity": torch.as_tensor(rng.normal(size=n)), "color": torch.as_tensor(rng.normal(size=(n, 48)))}


def test_activation_closed_forms():
    K = 8
    raw = {k: torch.zeros_like(v) for k, v in _raw(3, K, 0).items()}
    raw["q"][:, 0] = 2.0
    a = O.activate(raw)
    np.testing.assert_allclose(a["opacity"].numpy(), 0.5)
    np.testing.assert_allclose(a["eta"].numpy(), 0.5)
    np.testing.assert_allclose(a["tau"].numpy(), -0.1 + 1.09 * 0.5)
    np.testing.assert_allclose(a["scale"].numpy(), 1.0)
    np.testing.assert_allclose(a["q"].numpy(), np.tile([1.0, 0, 0, 0], (3, 1)))
    # equal raw angles: K equal sectors starting at 0
    np.testing.assert_allclose(a["theta"].numpy(), np.tile(2 * math.pi * np.arange(K) / K, (3, 1)), atol=1e-15)
    # tau's range: (-0.1, 0.99)
    t = O.activate({**raw, "tau": torch.tensor([-50.0, 50.0, 0.0])})["tau"].numpy()
    assert t[0] == pytest.approx(-0.1, abs=1e-12) and t[1] == pytest.approx(0.99, abs=1e-12)


@pytest.mark.parametrize("K", [3, 5, 8, 16])
def test_activated_angles_are_valid_for_any_raw_values(K):
    """theta_0 = 0, increasing, every gap (wrap included) below pi for raw values whose sigmoids do
    not round to 0 or 1.  The supremum of the largest gap is exactly pi for every K, reached only as
    one sigmoid -> 1 and the others -> 0: (1 + 1/(K-2)) / (1 + K/(K-2)) = 1/2 of the turn."""
    for spread in (1.0, 5.0):
        th = O.activate(_raw(500, K, K, spread))["theta"].numpy()
        gaps = np.diff(np.concatenate([th, np.full((th.shape[0], 1), 2 * math.pi)], 1), axis=1)
        assert (th[:, 0] == 0).all() and (gaps > 0).all() and (gaps < math.pi).all()
    raw = {k: v[:1] for k, v in _raw(1, K, 1).items()}
    raw["theta"] = torch.full((1, K), -60.0, dtype=torch.float64)
    raw["theta"][0, 2] = 60.0
    g = np.diff(np.concatenate([O.activate(raw)["theta"].numpy()[0], [2 * math.pi]]))
    assert 2 * math.pi * (1 + 1 / (K - 2)) / (1 + K / (K - 2)) == pytest.approx(math.pi, rel=1e-15)
    assert g.max() == pytest.approx(math.pi, rel=1e-12)


def test_activation_vjp_against_central_differences():
    raw = _raw(4, 5, 3)
    rng = np.random.default_rng(4)
    g_act = {k: torch.as_tensor(rng.normal(size=v.shape)) for k, v in raw.items()}
    grads = O.activate_vjp(raw, g_act)
    f = lambda r: sum(float((O.activate(r)[k] * g_act[k]).sum()) for k in g_act)
    h = 1e-6
    for k in raw:
        flat = raw[k].reshape(-1)
        for i in range(0, flat.numel(), max(1, flat.numel() // 6)):
            rp = {kk: vv.clone() for kk, vv in raw.items()}
            rm = {kk: vv.clone() for kk, vv in raw.items()}
            rp[k].reshape(-1)[i] += h
            rm[k].reshape(-1)[i] -= h
            fd = (f(rp) - f(rm)) / (2 * h)
            assert float(grads[k].reshape(-1)[i]) == pytest.approx(fd, rel=1e-6, abs=1e-8), (k, i)


def test_adam_first_step_and_fixed_point():
    """At step 1 the bias-corrected update is lr * g / (|g| + eps): each parameter moves by lr
    against the sign of its gradient; with zero gradient and zero moments nothing moves."""
    g = np.array([3.0, -0.2, 1e-3, 0.0])
    p, m, v = O.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 0.01, 0.9, 0.999, 1e-15, 1)
    np.testing.assert_allclose(p, [-0.01, 0.01, -0.01, 0.0], rtol=1e-9)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
    # two steps with a constant gradient: the update stays lr * sign(g) (m_hat = g, v_hat = g^2)
    p2, _, _ = O.adam_step(p, m, v, g, 0.01, 0.9, 0.999, 1e-15, 2)
    np.testing.assert_allclose(p2, 2 * p, rtol=1e-9)


# ---- Sec. 3.1 (3D-GS rotation of a quaternion q = (w, x, y, z)): R(q) against scipy's rotation
#      matrix, against Rodrigues' formula for a known axis and angle, and a hand-checked 90 degree
#      turn.  The columns of R are the local u axis, v axis and plane normal in world coordinates.
def test_quaternion_rotation_against_scipy_and_rodrigues():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(21)
    q = rng.normal(size=(64, 4))
    q[0] = [3.0, 0.0, 0.0, 0.0]                    # not unit length: normalised first
    R = O.quat_to_rotmat(_t(q)).numpy()
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()   # scipy takes (x, y, z, w)
    np.testing.assert_allclose(R, ref, atol=1e-14)
    # Rodrigues: rotation by angle a about unit axis k is I + sin(a) [k]x + (1 - cos(a)) [k]x^2,
    # and the unit quaternion of that rotation is (cos(a/2), sin(a/2) k)
    for _ in range(16):
        k = rng.normal(size=3)
        k /= np.linalg.norm(k)
        a = rng.uniform(-math.pi, math.pi)
        Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        Rr = np.eye(3) + math.sin(a) * Kx + (1 - math.cos(a)) * (Kx @ Kx)
        qa = np.concatenate([[math.cos(a / 2)], math.sin(a / 2) * k]) * rng.uniform(0.5, 2.0)
        np.testing.assert_allclose(O.quat_to_rotmat(_t(qa)).numpy(), Rr, atol=1e-14)
    # 90 degrees about +z: the local u axis goes to world +y, v to world -x, the normal stays +z
    h = math.sqrt(0.5)
    R90 = O.quat_to_rotmat(_t([h, 0.0, 0.0, h])).numpy()
    np.testing.assert_allclose(R90[:, 0], [0, 1, 0], atol=1e-15)
    np.testing.assert_allclose(R90[:, 1], [-1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(R90[:, 2], [0, 0, 1], atol=1e-15)


def _lowpass_scene(mu, q, s, o, col, K=4):
    """One DRK with equal basis lengths s on axis-aligned angles, eta = tau = 0, RGB colour."""
    return Scene(np.asarray(mu, np.float32).reshape(3, 1), np.asarray(q, np.float32).reshape(4, 1),
                 np.full((K, 1), s, np.float32),
                 (np.arange(K, dtype=np.float64) * 2 * math.pi / K).astype(np.float32).reshape(K, 1),
                 np.zeros(1, np.float32), np.zeros(1, np.float32), np.array([o], np.float32),
                 np.asarray(col, np.float32).reshape(3, 1), -1)


def _lowpass_closed_form(mu, q, o, sl, cam, alpha_kernel=None):
    """The Sec. 4.4 low-pass term written out from the camera geometry:
    f = o exp(-|p - p_c|^2 / (2 s_l^2 cos^2)), p_c the pinhole projection of the centre, cos the
    cosine between the unit pixel ray and the plane normal.  The normal is the third column of the
    rotation by angle a about axis k, read off the float32 quaternion as (cos(a/2), sin(a/2) k),
    through Rodrigues' formula."""
    q = np.asarray(q, np.float32).astype(np.float64)
    q = q / np.linalg.norm(q)
    sv = np.linalg.norm(q[1:])
    if sv > 0:
        k, angle = q[1:] / sv, 2.0 * math.atan2(sv, q[0])
    else:
        k, angle = np.array([1.0, 0.0, 0.0]), 0.0
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    n = (np.eye(3) + math.sin(angle) * Kx + (1 - math.cos(angle)) * (Kx @ Kx))[:, 2]
    H, W = cam.height, cam.width
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    m = np.asarray(mu, np.float32).astype(np.float64)
    pcx, pcy = fx * m[0] / m[2] + cx, fy * m[1] / m[2] + cy
    yy, xx = np.mgrid[0:H, 0:W]
    X, Y = xx + 0.5, yy + 0.5
    ray = np.stack([(X - cx) / fx, (Y - cy) / fy, np.ones_like(X)], -1)      # camera = world here
    cos = np.abs(ray @ n) / np.linalg.norm(ray, axis=-1)
    sl32 = float(np.float32(sl))
    o32 = float(np.float32(o))
    f = o32 * np.exp(-((X - pcx) ** 2 + (Y - pcy) ** 2) / (2.0 * sl32 ** 2 * cos ** 2))
    a = f if alpha_kernel is None else np.maximum(alpha_kernel, f)
    return np.minimum(a, float(np.float32(0.99))).ravel()


# ---- Sec. 4.4 low-pass filter: a DRK whose kernel is far below one pixel contributes only the
#      low-pass term, so the image is f c + (1 - f) bg with f from the camera geometry (the
#      projected centre, |r_d . R_z| with r_d normalised, the square of that cosine, o outside
#      the exponential).  Fronto-parallel and tilted planes, centre off the optical axis.
@pytest.mark.parametrize("angle_deg", [0.0, 50.0, -35.0])
def test_lowpass_closed_form_tiny_primitive(angle_deg):
    W, H = 40, 32
    fx, fy, cx, cy = intrinsics_hfov(W, H, 60.0)
    bg = np.array([0.1, 0.2, 0.3], np.float32)
    cam = Camera(W, H, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.zeros(3, np.float32), bg)
    mu = [0.31, -0.17, 2.5]
    axis = [1.0, 0.4, 0.0]
    ang = math.radians(angle_deg)
    qa = [math.cos(ang / 2)] + list(math.sin(ang / 2) * np.asarray(axis) / np.linalg.norm(axis))
    col = np.array([0.9, 0.4, 0.1])
    o, sl = 0.8, 1.3                        # a wide filter so that many pixels see it
    sc = _lowpass_scene(mu, qa, 1e-5, o, col)
    opts = O.Opts(lowpass_sl=sl)
    r = O.render_image(sc, cam, opts)
    a = _lowpass_closed_form(mu, qa, o, sl, cam)
    a = np.where(a >= float(np.float32(1 / 255)), a, 0.0)
    ref = a[:, None] * col.astype(np.float32).astype(np.float64)[None] + (1 - a)[:, None] * bg.astype(np.float64)[None]
    assert (a > 0).sum() > 20
    np.testing.assert_allclose(r.rgb, ref, atol=1e-12)
    np.testing.assert_allclose(r.T, 1 - a, atol=1e-12)


# ---- Sec. 4.4: the low-pass value competes with the kernel's opacity after opacity and Psi are
#      applied: alpha~ = max(o Psi(g), f).  A fronto-parallel DRK in the Gaussian case of Sec. 4.1
#      (eta = 0, lengths (s_u, s_v, s_u, s_v) on the axes): long along u, where the kernel wins,
#      and thin along v, where the filter wins.  tau = 0 makes Psi the identity (its three pieces
#      all have slope 1 and meet at g = 1/4 and 3/4).
def test_lowpass_max_against_the_kernel():
    W, H = 48, 40
    fx, fy, cx, cy = intrinsics_hfov(W, H, 60.0)
    cam = Camera(W, H, fx, fy, cx, cy, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))
    d, su, sv, o, sl = 3.0, 0.3, 0.03, 0.7, 0.9
    mu = [0.05, 0.02, d]
    sc = _lowpass_scene(mu, [1, 0, 0, 0], 1.0, o, [1.0, 1.0, 1.0])
    sc.scale[:, 0] = np.array([su, sv, su, sv], np.float32)
    r = O.render_image(sc, cam, O.Opts(lowpass_sl=sl))
    yy, xx = np.mgrid[0:H, 0:W]
    fx32, fy32, cx32, cy32 = (float(np.float32(v)) for v in (fx, fy, cx, cy))
    m = np.asarray(mu, np.float32).astype(np.float64)
    # the plane z = d is hit at (d (x - cx)/fx, d (y - cy)/fy); u, v are offsets from the centre
    u = d * (xx + 0.5 - cx32) / fx32 - m[0]
    v = d * (yy + 0.5 - cy32) / fy32 - m[1]
    su32, sv32, o32 = (float(np.float32(x)) for x in (su, sv, o))
    kern = o32 * np.exp(-0.5 * (u ** 2 / su32 ** 2 + v ** 2 / sv32 ** 2))
    a = _lowpass_closed_form(mu, [1, 0, 0, 0], o, sl, cam, alpha_kernel=kern)
    a = np.where(a >= float(np.float32(1 / 255)), a, 0.0)
    f_only = _lowpass_closed_form(mu, [1, 0, 0, 0], o, sl, cam)
    kern = kern.ravel()
    assert ((kern > f_only) & (a > 0)).sum() > 10 and ((f_only > kern) & (a > 0)).sum() > 10   # both branches
    # 1e-6: the float32 basis angles are pi/2 multiples only to 4e-8, which moves the kernel's
    # Gaussian reduction by ~2e-7 where it wins; a misplaced o, cosine or centre is off by > 1e-2
    np.testing.assert_allclose(r.T, 1 - a, atol=1e-6)
