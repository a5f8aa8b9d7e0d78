"""FP64 CPU oracle for the Deformable Radial Kernel (DRK) rasterizer.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library (``paper_2412_11752_amd``) and imports nothing from it.

Everything is computed per pixel over every primitive, in float64, from float32
inputs promoted exactly.  The method is defined by the paper (arXiv 2412.11752,
"Deformable Radial Kernel Splatting"); each function names the passage it
follows.  Where the paper is silent or garbled the oracle takes the readings
listed below (and in the design notes):

  * local axes t_u, t_v and normal n are the COLUMNS of R(q), q = (w, x, y, z)
    (Sec. 3.3 says "rows", which contradicts R_z being the normal);
  * polar angle theta = atan2(v, u) mod 2*pi (Sec. 4.1 prints arccos, which only
    covers [0, pi]); K angles ascending in [0, 2*pi), the last sector wraps
    from theta_{K-1} to theta_0 + 2*pi, and theta_k < theta <= theta_{k+1};
  * Sec. 4.4 low-pass: s_l = sqrt(2)/2 px, r_d normalised, the max is taken
    after opacity and sharpening;
  * cutoffs as in 3D-GS: alpha_min = 1/255, alpha_max = 0.99, T_min = 1e-4,
    a contribution whose transmittance would drop below T_min stops the pixel
    without being added; near plane 0.2;
  * cache sorting (Sec. 4.4 and Algorithm 1 of the supplement): only
    contributors enter a cache of L slots kept sorted by r_t (a newcomer goes
    after equal keys); when the cache is full its head is emitted BEFORE the
    newcomer is inserted; at the end of the list the cache drains from the
    head.  The arrival order is the pre-sort by (float32 key, primitive
    index), the key being the view-space depth of the centre, or one of the
    per-tile keys of ``tile_key`` (supplement, cache-sorting evaluation);
  * colour: real spherical harmonics of degree <= 3 at the direction from the
    camera to the centre, plus 0.5, clamped at 0 (3D-GS convention); a plain
    RGB colour is used as is;
  * background added with the final transmittance.

Parity unpinned: the low-pass radius s_l, the cutoff constants and the cache
semantics above have no numeric example in the paper; they are fixed by the
readings only.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

F64 = torch.float64
TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class Opts:
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    near: float = 0.2
    lowpass_sl: float = math.sqrt(0.5)   # 0 disables the low-pass filter
    cache_len: int = 8                   # >= 1<<30 means exact per-pixel sort
    cull_mode: int = 0                   # 0 conservative polygon, 1 paper polygon, 2 all tiles
    key_mode: int = 0                    # pre-sort key: 0 centre depth, 1 most centric, 2 nearest (per tile)

    def f32(self) -> "Opts":
        """The same options rounded to float32, as the C ABI carries them."""
        r = lambda x: float(np.float32(x))
        return Opts(r(self.alpha_min), r(self.alpha_max), r(self.T_min), r(self.near), r(self.lowpass_sl),
                    self.cache_len, self.cull_mode, self.key_mode)


EXACT = 1 << 30
GRAZING = 1e-6


def _f64(a) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a, dtype=np.float32).astype(np.float64))


# ---------------------------------------------------------------------------------------------
# Elementary pieces

def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of a (not necessarily unit) quaternion (w, x, y, z), as in 3D-GS (Sec. 3.1).
    Returns (..., 3, 3); columns are the primitive's local u axis, v axis and plane normal."""
    q = q / torch.linalg.vector_norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    rows = [
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ]
    return torch.stack(rows, -1).reshape(q.shape[:-1] + (3, 3))


def psi(g, tau):
    """Edge-sharpening remap (Sec. 4.3): piecewise linear in g with breakpoints (1+tau)/4 and (3-tau)/4."""
    lo = (1 + tau) / 4
    hi = (3 - tau) / 4
    flat = (1 - tau) / (1 + tau)
    steep = (1 + tau) / (1 - tau)
    p1 = flat * g
    p2 = steep * g - tau / (1 - tau)
    p3 = flat * g + 2 * tau / (1 + tau)
    return torch.where(g < lo, p1, torch.where(g < hi, p2, p3))


def psi_inv(y, tau):
    """Inverse of ``psi`` (the three pieces inverted; the image breakpoints are (1-tau)/4 and (3+tau)/4)."""
    y = torch.as_tensor(y, dtype=F64)
    tau = torch.as_tensor(tau, dtype=F64)
    p1 = y * (1 + tau) / (1 - tau)
    p2 = (y * (1 - tau) + tau) / (1 + tau)
    p3 = (y * (1 + tau) - 2 * tau) / (1 - tau)
    return torch.where(y < (1 - tau) / 4, p1, torch.where(y < (3 + tau) / 4, p2, p3))


_SQ = math.sqrt
_PI = math.pi


def real_sh(deg: int, d: torch.Tensor) -> torch.Tensor:
    """Real spherical harmonics Y_{l,m}, l <= deg, of unit directions d (..., 3); index l*l + l + m.
    Standard orthonormal real basis (Cartesian polynomial forms)."""
    x, y, z = d.unbind(-1)
    out = [torch.full_like(x, 0.5 / _SQ(_PI))]
    if deg >= 1:
        c1 = _SQ(3.0 / (4 * _PI))
        out += [c1 * y, c1 * z, c1 * x]
    if deg >= 2:
        out += [0.5 * _SQ(15.0 / _PI) * x * y,
                0.5 * _SQ(15.0 / _PI) * y * z,
                0.25 * _SQ(5.0 / _PI) * (3 * z * z - 1),
                0.5 * _SQ(15.0 / _PI) * x * z,
                0.25 * _SQ(15.0 / _PI) * (x * x - y * y)]
    if deg >= 3:
        out += [0.25 * _SQ(35.0 / (2 * _PI)) * y * (3 * x * x - y * y),
                0.5 * _SQ(105.0 / _PI) * x * y * z,
                0.25 * _SQ(21.0 / (2 * _PI)) * y * (5 * z * z - 1),
                0.25 * _SQ(7.0 / _PI) * (5 * z * z * z - 3 * z),
                0.25 * _SQ(21.0 / (2 * _PI)) * x * (5 * z * z - 1),
                0.25 * _SQ(105.0 / _PI) * z * (x * x - y * y),
                0.25 * _SQ(35.0 / (2 * _PI)) * x * (x * x - 3 * y * y)]
    return torch.stack(out, -1)


def drk_energy(u, v, s, theta, eta):
    """E = eta * r1^2 + (1 - eta) * r2^2 / sbar^2 (Sec. 4.1 radial basis + Sec. 4.2 L1 term).

    u, v: (L,) tangent coordinates; s, theta: (L, K) basis lengths and angles; eta: (L,).
    Returns (E, k) with k the sector index (theta_k < theta <= theta_{k+1}, wrapping)."""
    K = s.shape[-1]
    r2sq = u * u + v * v
    centre = r2sq == 0
    us = torch.where(centre, torch.ones_like(u), u)
    vs = torch.where(centre, torch.zeros_like(v), v)
    th = torch.remainder(torch.atan2(vs, us), TWO_PI)
    th = torch.where(th <= theta[:, 0], th + TWO_PI, th)
    k = (theta < th.detach()[:, None]).sum(-1) - 1
    kn = torch.remainder(k + 1, K)
    wrap = (k == K - 1).to(F64)
    th_k = theta.gather(-1, k[:, None]).squeeze(-1)
    th_n = theta.gather(-1, kn[:, None]).squeeze(-1) + TWO_PI * wrap
    s_k = s.gather(-1, k[:, None]).squeeze(-1)
    s_n = s.gather(-1, kn[:, None]).squeeze(-1)
    # Sec. 4.1: relative angular distance and cosine-interpolated inverse squared scale
    dtheta = math.pi * (th - th_k) / (th_n - th_k)
    inv_sbar2 = (1 + torch.cos(dtheta)) / (2 * s_k * s_k) + (1 - torch.cos(dtheta)) / (2 * s_n * s_n)
    # Sec. 4.2, L1 norm: solve [e_k e_{k+1}] (a, b)^T = (u, v)^T
    ekx, eky = s_k * torch.cos(th_k), s_k * torch.sin(th_k)
    enx, eny = s_n * torch.cos(th_n), s_n * torch.sin(th_n)
    det = ekx * eny - enx * eky
    a = (us * eny - vs * enx) / det
    b = (ekx * vs - eky * us) / det
    r1 = torch.abs(a) + torch.abs(b)
    E = eta * r1 * r1 + (1 - eta) * r2sq * inv_sbar2
    E = torch.where(centre, torch.zeros_like(E), E)
    return E, k


def drk_alpha_uv(u, v, s, theta, eta, tau, o):
    """alpha = o * Psi(g), g = exp(-E/2) (Sec. 4.2 Eq. kernel, Sec. 4.3)."""
    E, _ = drk_energy(u, v, s, theta, eta)
    return o * psi(torch.exp(-0.5 * E), tau)


# ---------------------------------------------------------------------------------------------
# Scene / camera containers in float64

@dataclasses.dataclass
class Prims:
    """Primitive parameters as (N, ...) float64 tensors (may require grad)."""
    mu: torch.Tensor      # (N, 3)
    q: torch.Tensor       # (N, 4)
    s: torch.Tensor       # (N, K)
    theta: torch.Tensor   # (N, K)
    eta: torch.Tensor     # (N,)
    tau: torch.Tensor     # (N,)
    o: torch.Tensor       # (N,)
    color: torch.Tensor   # (N, 3) RGB or (N, C, 3) SH coefficients
    sh_degree: int

    @staticmethod
    def from_scene(scene) -> "Prims":
        n = scene.n
        if scene.sh_degree < 0:
            col = _f64(scene.color).T.contiguous()
        else:
            nc = (scene.sh_degree + 1) ** 2
            col = _f64(scene.color).reshape(nc, 3, n).permute(2, 0, 1).contiguous()
        return Prims(_f64(scene.mu).T.contiguous(), _f64(scene.q).T.contiguous(),
                     _f64(scene.scale).T.contiguous(), _f64(scene.theta).T.contiguous(),
                     _f64(scene.eta), _f64(scene.tau), _f64(scene.opacity), col, scene.sh_degree)

    def index(self, idx) -> "Prims":
        return Prims(self.mu[idx], self.q[idx], self.s[idx], self.theta[idx], self.eta[idx], self.tau[idx],
                     self.o[idx], self.color[idx], self.sh_degree)


@dataclasses.dataclass
class Cam:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: torch.Tensor   # (3, 3) world -> camera
    t: torch.Tensor   # (3,)
    bg: torch.Tensor  # (3,)

    @staticmethod
    def from_camera(c) -> "Cam":
        f = lambda x: float(np.float32(x))
        return Cam(int(c.width), int(c.height), f(c.fx), f(c.fy), f(c.cx), f(c.cy),
                   _f64(c.R).reshape(3, 3), _f64(c.t).reshape(3), _f64(c.bg).reshape(3))

    @property
    def Rinv(self) -> torch.Tensor:
        """Camera-to-world rotation: the exact inverse of the world-to-camera R (X_c = R X_w + t).
        R is given in float32, so its transpose is only approximately its inverse."""
        return torch.linalg.inv(self.R)

    @property
    def position(self) -> torch.Tensor:
        return -(self.Rinv @ self.t)


# ---------------------------------------------------------------------------------------------
# Per primitive (view independent of the pixel)

def centre_depth_f32(mu: np.ndarray, cam) -> np.ndarray:
    """float32 view-space depth of each centre, computed in float64 as ((r20*x + r21*y) + r22*z) + t2
    and rounded once.  This is the global pre-sort key (3D-GS centre-depth order, Sec. 4.4)."""
    R = np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float32).astype(np.float64).reshape(3)
    m = np.asarray(mu, np.float32).astype(np.float64)
    z = R[2, 0] * m[0]
    z = z + R[2, 1] * m[1]
    z = z + R[2, 2] * m[2]
    z = z + t[2]
    return z.astype(np.float32)


def prim_colors(P: Prims, cam: Cam) -> torch.Tensor:
    """Per-primitive RGB: plain colour, or SH at the camera-to-centre direction + 0.5 clamped at 0."""
    if P.sh_degree < 0:
        return P.color
    d = P.mu - cam.position
    d = d / torch.linalg.vector_norm(d, dim=-1, keepdim=True)
    Y = real_sh(P.sh_degree, d)                        # (N, C)
    rgb = torch.einsum("nc,nck->nk", Y, P.color) + 0.5
    return torch.clamp(rgb, min=0.0)


def calibrated_radius(o, tau, alpha_min):
    """c such that {E <= c^2} is exactly {o * Psi(g) >= alpha_min} (corrected Eq. calibrate, Sec. 4.4):
    c = sqrt(-2 ln Psi^{-1}(alpha_min / o))."""
    g_min = psi_inv(torch.as_tensor(alpha_min, dtype=F64) / o, tau)
    return torch.sqrt(-2.0 * torch.log(g_min))


def culled_mask(P: Prims, cam: Cam, opts: Opts) -> torch.Tensor:
    """Primitives that can never contribute: centre at or behind the near plane, opacity below
    alpha_min, or invalid parameters."""
    zc = (P.mu @ cam.R.T + cam.t)[:, 2]
    th = P.theta
    gaps = torch.diff(torch.cat([th, th[:, :1] + TWO_PI], 1), dim=1)
    bad = ~torch.isfinite(P.mu).all(-1) | ~torch.isfinite(P.q).all(-1) | ~torch.isfinite(P.s).all(-1) \
        | (P.s <= 0).any(-1) | (th < 0).any(-1) | (th >= TWO_PI).any(-1) | (gaps <= 0).any(-1) \
        | (gaps >= math.pi).any(-1) | (P.o <= 0) | (P.o > 1) | (P.tau <= -1) | (P.tau >= 1) \
        | (P.eta < 0) | (P.eta > 1)
    return (zc <= opts.near) | (P.o < opts.alpha_min) | bad


# ---------------------------------------------------------------------------------------------
# Per (pixel, primitive) pair: ray-plane hit (Sec. 3.3), kernel, low-pass (Sec. 4.4)

def pixel_rays(cam: Cam, px: torch.Tensor, py: torch.Tensor):
    """Unit world-space ray directions through pixel centres (px + 0.5, py + 0.5)."""
    dc = torch.stack([(px.to(F64) + 0.5 - cam.cx) / cam.fx, (py.to(F64) + 0.5 - cam.cy) / cam.fy,
                      torch.ones_like(px, dtype=F64)], -1)
    rd = dc @ cam.Rinv.T     # R^-1 dc for each row
    return rd / torch.linalg.vector_norm(rd, dim=-1, keepdim=True)


def eval_pairs(P: Prims, cam: Cam, opts: Opts, px: torch.Tensor, py: torch.Tensor, colors: torch.Tensor):
    """Evaluate alpha-tilde and r_t for pixel/primitive pairs.  ``P`` and ``colors`` are already
    gathered per pair (length L).  Returns a dict of (L,) tensors."""
    R = quat_to_rotmat(P.q)                       # (L, 3, 3)
    tu, tv, n = R[..., 0], R[..., 1], R[..., 2]
    ro = cam.position
    rd = pixel_rays(cam, px, py)                  # (L, 3)
    den = (rd * n).sum(-1)                        # r_d . R_z
    ok = den.abs() >= GRAZING
    den_s = torch.where(ok, den, torch.ones_like(den))
    rt = ((P.mu - ro) * n).sum(-1) / den_s        # Sec. 4.4 Cache Sorting: r_t
    zc = rt * (rd @ cam.R[2])                     # view depth of the hit
    ok = ok & (zc > opts.near)
    hit = ro + rt[:, None] * rd                   # Sec. 3.3 intersection point
    u = ((hit - P.mu) * tu).sum(-1)
    v = ((hit - P.mu) * tv).sum(-1)
    alpha = drk_alpha_uv(u, v, P.s, P.theta, P.eta, P.tau, P.o)
    if opts.lowpass_sl > 0:
        mc = P.mu @ cam.R.T + cam.t
        pxc = cam.fx * mc[:, 0] / mc[:, 2] + cam.cx
        pyc = cam.fy * mc[:, 1] / mc[:, 2] + cam.cy
        d2 = (px.to(F64) + 0.5 - pxc) ** 2 + (py.to(F64) + 0.5 - pyc) ** 2
        f = P.o * torch.exp(-d2 / (2.0 * den_s * den_s * opts.lowpass_sl ** 2))
        at = torch.maximum(alpha, f)
    else:
        at = alpha
    at = torch.clamp(at, max=opts.alpha_max)
    contrib = ok & (at >= opts.alpha_min)
    # unit normal of the plane in the camera frame (the image of the plane under X -> R X + t),
    # turned toward the camera: n_c . mu_c < 0
    a = torch.linalg.cross(tu @ cam.R.T, tv @ cam.R.T)
    a = a / torch.linalg.vector_norm(a, dim=-1, keepdim=True)
    side = ((P.mu @ cam.R.T + cam.t) * a).sum(-1)
    nc = torch.where((side > 0)[:, None], -a, a)
    return dict(alpha=at, rt=rt, zc=zc, den=den, ok=ok, contrib=contrib, u=u, v=v, color=colors, normal=nc)


# ---------------------------------------------------------------------------------------------
# Candidate prefilter (lossless): every contributing hit lies in the ball of radius c*max_k s_k
# around the centre (both the L1 chord and sbar are bounded by the larger endpoint length) and in
# front of the near plane; the low-pass term needs the pixel within s_l*sqrt(2 ln(o/alpha_min)).

def screen_bounds(P: Prims, cam: Cam, opts: Opts) -> Tuple[torch.Tensor, torch.Tensor]:
    """Conservative pixel-space boxes (N, 4) = (x0, x1, y0, y1) of the possible support, and the
    culled mask."""
    with torch.no_grad():
        cull = culled_mask(P, cam, opts)
        o = torch.clamp(P.o, min=opts.alpha_min)
        c = calibrated_radius(o, P.tau, opts.alpha_min)
        rho = c * P.s.max(-1).values
        mc = P.mu @ cam.R.T + cam.t
        X, Y, Z = mc.unbind(-1)
        zlo = torch.clamp(Z - rho, min=opts.near)
        zhi = Z + rho
        inv = lambda a, b: (a / b)
        xs = torch.stack([inv(X - rho, zlo), inv(X - rho, zhi), inv(X + rho, zlo), inv(X + rho, zhi)], -1)
        ys = torch.stack([inv(Y - rho, zlo), inv(Y - rho, zhi), inv(Y + rho, zlo), inv(Y + rho, zhi)], -1)
        box = torch.stack([cam.fx * xs.min(-1).values + cam.cx, cam.fx * xs.max(-1).values + cam.cx,
                           cam.fy * ys.min(-1).values + cam.cy, cam.fy * ys.max(-1).values + cam.cy], -1)
        if opts.lowpass_sl > 0:
            rl = opts.lowpass_sl * torch.sqrt(2.0 * torch.log(torch.clamp(o / opts.alpha_min, min=1.0)))
            pxc = cam.fx * X / Z + cam.cx
            pyc = cam.fy * Y / Z + cam.cy
            box = torch.stack([torch.minimum(box[:, 0], pxc - rl), torch.maximum(box[:, 1], pxc + rl),
                               torch.minimum(box[:, 2], pyc - rl), torch.maximum(box[:, 3], pyc + rl)], -1)
        pad = 1e-3 + 1e-9 * box.abs()
        box = box + torch.stack([-pad[:, 0], pad[:, 1], -pad[:, 2], pad[:, 3]], -1)
        cull = cull | (zhi <= opts.near)
    return box, cull


# ---------------------------------------------------------------------------------------------
# Ordering: Algorithm 1 (cache sorting) and the exact sort

def cache_emit(seq: Sequence[Tuple[float, int]], L: int) -> List[Tuple[float, int]]:
    """Emission order of a pixel's contributors arriving in ``seq`` order through an L-slot cache
    sorted by r_t (Algorithm 1 of the supplement, reading: a full cache emits its head before the
    newcomer is inserted; newcomers go after equal keys; the remainder drains from the head)."""
    return cache_trace(seq, L)[0]


def cache_trace(seq: Sequence[Tuple[float, int]], L: int):
    """``cache_emit`` plus, for knife-edge detection: for each emission the number of arrivals seen
    when it was emitted, and for each arrival the smallest relative key gap to the cache entries it
    was compared with on insertion."""
    cache: List[Tuple[float, int]] = []
    out: List[Tuple[float, int]] = []
    at: List[int] = []
    gaps: List[float] = []
    for i, (rt, j) in enumerate(seq):
        if len(cache) >= L:
            out.append(cache.pop(0))
            at.append(i + 1)
        g = min((abs(rt - c[0]) / max(abs(rt), 1e-300) for c in cache), default=math.inf)
        gaps.append(g)
        pos = len(cache)
        while pos > 0 and cache[pos - 1][0] > rt:
            pos -= 1
        cache.insert(pos, (rt, j))
    out.extend(cache)
    at.extend([len(seq)] * len(cache))
    return out, at, gaps


def composite(alphas: Sequence[float], cols: Sequence[Sequence[float]], bg, T_min):
    """Front-to-back alpha blending, Eq. (1): C = sum_i T_i alpha_i c_i + T_final * bg.  A contribution
    whose resulting transmittance would fall below T_min ends the pixel without being added."""
    T = 1.0
    C = [0.0, 0.0, 0.0]
    n = 0
    weights = []
    for a, c in zip(alphas, cols):
        test = T * (1.0 - a)
        if test < T_min:
            break
        w = T * a
        for ch in range(3):
            C[ch] += w * c[ch]
        weights.append(w)
        T = test
        n += 1
    for ch in range(3):
        C[ch] += T * float(bg[ch])
    return C, T, n, weights


# ---------------------------------------------------------------------------------------------
# Full per-pixel renderer

@dataclasses.dataclass
class PixelResult:
    rgb: np.ndarray          # (P, 3)
    T: np.ndarray            # (P,)
    n_emit: np.ndarray       # (P,) int
    n_contrib: np.ndarray    # (P,) int
    knife: np.ndarray        # (P,) bool: some decision within 1e-6 (relative) of its threshold
    emitted: List[List[int]]  # per pixel, primitive indices actually composited, in order
    weights: List[List[float]]
    emitted_z: List[List[float]]  # per pixel, view depth of the hit of each composited contribution
    depth: np.ndarray = None  # (P,) sum over composited contributions of T_i alpha_i * view depth of the hit
    normal: np.ndarray = None  # (P, 3) sum of T_i alpha_i * unit camera-frame normal facing the camera


def render_pixels(scene, camera, opts: Opts, px: np.ndarray, py: np.ndarray, chunk: int = 64,
                  prims: Optional[Prims] = None, prefilter: bool = True,
                  tile_members: Optional[Dict[int, set]] = None) -> PixelResult:
    """Render the given pixel centres by testing every primitive (through the lossless prefilter
    unless ``prefilter`` is False).  With ``tile_members`` (tile id -> set of primitive ids) only the
    primitives binned to the pixel's tile are considered, to show that binning changes nothing."""
    P = prims if prims is not None else Prims.from_scene(scene)
    cam = Cam.from_camera(camera)
    akey = arrival_keys(scene, camera, opts, np.asarray(px), np.asarray(py))
    with torch.no_grad():
        box, cull = screen_bounds(P, cam, opts)
        colors = prim_colors(P, cam)
        alive = torch.nonzero(~cull).squeeze(-1)
        box_a = box[alive]
        px_t = torch.as_tensor(np.asarray(px), dtype=torch.int64)
        py_t = torch.as_tensor(np.asarray(py), dtype=torch.int64)
        npix = px_t.numel()
        out_rgb = np.zeros((npix, 3))
        out_T = np.ones(npix)
        out_n = np.zeros(npix, np.int64)
        out_nc = np.zeros(npix, np.int64)
        knife = np.zeros(npix, bool)
        emitted: List[List[int]] = [[] for _ in range(npix)]
        weights: List[List[float]] = [[] for _ in range(npix)]
        emitted_z: List[List[float]] = [[] for _ in range(npix)]
        out_depth = np.zeros(npix)
        out_normal = np.zeros((npix, 3))
        bg = cam.bg.numpy()
        for c0 in range(0, npix, chunk):
            cx_ = px_t[c0:c0 + chunk].to(F64)[:, None] + 0.5
            cy_ = py_t[c0:c0 + chunk].to(F64)[:, None] + 0.5
            if prefilter:
                inside = (cx_ >= box_a[None, :, 0]) & (cx_ <= box_a[None, :, 1]) & \
                         (cy_ >= box_a[None, :, 2]) & (cy_ <= box_a[None, :, 3])
            else:
                inside = torch.ones(cx_.shape[0], alive.numel(), dtype=torch.bool)
            if tile_members is not None:
                tx = (cam.width + TILE - 1) // TILE
                tid = (py_t[c0:c0 + chunk] // TILE) * tx + px_t[c0:c0 + chunk] // TILE
                alive_l = alive.tolist()
                mem = torch.zeros_like(inside)
                for r, t in enumerate(tid.tolist()):
                    members = tile_members.get(t, set())
                    mem[r] = torch.tensor([a in members for a in alive_l], dtype=torch.bool)
                inside = inside & mem
            pl, ml = torch.nonzero(inside, as_tuple=True)
            pj = alive[ml]
            pidx = pl + c0
            res = eval_pairs(P.index(pj), cam, opts, px_t[pidx], py_t[pidx], colors[pj])
            _finish_pixels(res, pidx, pj, akey, opts, bg, out_rgb, out_T, out_n, out_nc, knife, emitted, weights,
                           emitted_z, c0, min(chunk, npix - c0), out_depth, out_normal)
    return PixelResult(out_rgb, out_T, out_n, out_nc, knife, emitted, weights, emitted_z, out_depth, out_normal)


def _near(x, thr, rel=1e-6):
    return np.abs(x - thr) <= rel * abs(thr)


def _finish_pixels(res, pidx, pj, akey, opts, bg, out_rgb, out_T, out_n, out_nc, knife, emitted, weights,
                   emitted_z, c0, cnt, out_depth, out_normal):
    contrib = res["contrib"].numpy()
    ok = res["ok"].numpy()
    at = res["alpha"].numpy()
    rt = res["rt"].numpy()
    zc = res["zc"].numpy()
    den = res["den"].numpy()
    col = res["color"].numpy()
    nrm = res["normal"].numpy()
    pidx = pidx.numpy()
    pj = pj.numpy()
    # knife-edge decisions (value within 1e-6 relative of a threshold)
    edge = (_near(at, opts.alpha_min) & ok) | _near(np.abs(den), GRAZING) | _near(zc, opts.near)
    order = np.argsort(pidx, kind="stable")
    pidx_s = pidx[order]
    bounds = np.searchsorted(pidx_s, np.arange(c0, c0 + cnt + 1))
    for i in range(cnt):
        sel = order[bounds[i]:bounds[i + 1]]
        p = c0 + i
        if edge[sel].any():
            knife[p] = True
        sel = sel[contrib[sel]]
        out_nc[p] = sel.size
        if sel.size == 0:
            out_rgb[p] = bg
            continue
        if opts.cache_len >= EXACT:
            em = sorted(((float(rt[s]), int(pj[s])) for s in sel))
            emit_at = list(range(1, len(em) + 1))
            gaps = [math.inf] + [abs(em[i][0] - em[i - 1][0]) / abs(em[i][0]) for i in range(1, len(em))]
        else:
            arrival = sorted(sel, key=lambda s: (akey(p, int(pj[s])), int(pj[s])))
            em, emit_at, gaps = cache_trace([(float(rt[s]), int(pj[s])) for s in arrival], opts.cache_len)
        lut = {int(pj[s]): s for s in sel}
        em_s = [lut[j] for _, j in em]
        C, T, n, w = composite([at[s] for s in em_s], [col[s] for s in em_s], bg, opts.T_min)
        # knife edge on the stopping test: T*(1-a) within 1e-6 of T_min for any tested step
        Tt = 1.0
        for s in em_s[:n + 1]:
            test = Tt * (1 - at[s])
            if _near(test, opts.T_min):
                knife[p] = True
            Tt = test
        # order knife edge: a key comparison made before the pixel stopped was within 1e-6
        last = emit_at[min(n, len(emit_at) - 1)]
        if any(g <= 1e-6 for g in gaps[:last]):
            knife[p] = True
        out_rgb[p] = C
        out_T[p] = T
        out_n[p] = n
        emitted[p] = [int(pj[s]) for s in em_s[:n]]
        emitted_z[p] = [float(zc[s]) for s in em_s[:n]]
        weights[p] = w
        out_depth[p] = sum(wi * zc[s] for wi, s in zip(w, em_s))
        out_normal[p] = np.sum([wi * nrm[s] for wi, s in zip(w, em_s)], axis=0) if n else 0.0


def render_image(scene, camera, opts: Opts, **kw) -> PixelResult:
    H, W = camera.height, camera.width
    yy, xx = np.mgrid[0:H, 0:W]
    return render_pixels(scene, camera, opts, xx.ravel(), yy.ravel(), **kw)


# ---------------------------------------------------------------------------------------------
# Differentiable render of given pixels with the emission order fixed by the forward pass

def render_loss_grad(scene, camera, opts: Opts, px: np.ndarray, py: np.ndarray, target: np.ndarray,
                     dL_drgb: Optional[np.ndarray] = None, fwd: Optional[PixelResult] = None):
    """Gradients of L = sum over the pixels of (C - target)^2 (or of sum(C * dL_drgb) when given)
    with respect to every ABI parameter, by float64 autograd through Sec. 3.3 - 4.4 with the discrete
    decisions (emission order, cutoffs, sector, Psi piece, max branch) taken from the forward pass."""
    if fwd is None:
        fwd = render_pixels(scene, camera, opts, px, py)
    P = Prims.from_scene(scene)
    leaves = {}
    for name in ("mu", "q", "s", "theta", "eta", "tau", "o", "color"):
        t = getattr(P, name).clone().requires_grad_(True)
        leaves[name] = t
        setattr(P, name, t)
    cam = Cam.from_camera(camera)
    pix_l, prim_l, slot_l = [], [], []
    npix = len(px)
    maxE = max([len(e) for e in fwd.emitted] + [1])
    for p, em in enumerate(fwd.emitted):
        for k, j in enumerate(em):
            pix_l.append(p)
            prim_l.append(j)
            slot_l.append(k)
    pix_i = torch.as_tensor(pix_l, dtype=torch.int64)
    prim_i = torch.as_tensor(prim_l, dtype=torch.int64)
    slot_i = torch.as_tensor(slot_l, dtype=torch.int64)
    colors = prim_colors(P, cam)
    pxt = torch.as_tensor(np.asarray(px), dtype=torch.int64)
    pyt = torch.as_tensor(np.asarray(py), dtype=torch.int64)
    if prim_i.numel():
        res = eval_pairs(P.index(prim_i), cam, opts, pxt[pix_i], pyt[pix_i], colors[prim_i])
        A = torch.zeros(npix, maxE, dtype=F64).index_put((pix_i, slot_i), res["alpha"])
        Cc = torch.zeros(npix, maxE, 3, dtype=F64).index_put((pix_i, slot_i), res["color"])
    else:
        A = torch.zeros(npix, maxE, dtype=F64)
        Cc = torch.zeros(npix, maxE, 3, dtype=F64)
    one_minus = 1 - A
    T_incl = torch.cumprod(one_minus, dim=1)
    T_excl = torch.cat([torch.ones(npix, 1, dtype=F64), T_incl[:, :-1]], 1)
    rgb = (T_excl[..., None] * A[..., None] * Cc).sum(1) + T_incl[:, -1:] * cam.bg
    if dL_drgb is None:
        tgt = torch.as_tensor(np.asarray(target, np.float64))
        loss = ((rgb - tgt) ** 2).sum()
    else:
        loss = (rgb * torch.as_tensor(np.asarray(dL_drgb, np.float64))).sum()
    loss.backward()
    grads = {k: (v.grad if v.grad is not None else torch.zeros_like(v)).detach() for k, v in leaves.items()}
    return float(loss.detach()), grads, rgb.detach().numpy(), fwd


# ---------------------------------------------------------------------------------------------
# Kernel culling: conservative support polygon and tile lists (Sec. 4.4 Kernel Culling)

TILE = 16


def support_polygon(s: np.ndarray, theta: np.ndarray, c: float) -> np.ndarray:
    """Star polygon (6K, 2) in tangent coordinates that contains {E <= c^2}.

    E is a convex combination of r1^2 and r2^2/sbar^2, so E <= c^2 implies r1 <= c or r2 <= c*sbar:
    along a direction theta the support reaches at most c * max(chord(theta), sbar(theta)), with
    chord(theta) the distance to the segment e_k e_{k+1} (Eq. L1 level set) and sbar from Eq. radial.
    Within a sector sbar is monotone and chord = d / cos(theta - theta_p) is convex, so on each half
    of the sector [theta_k, mid] and [mid, theta_{k+1}] the larger bound is attained at an end.  At
    theta_k both equal s_k, at theta_{k+1} both equal s_{k+1}, and at the bisector (cos Delta = 0)
        sbar = (1/(2 s_k^2) + 1/(2 s_{k+1}^2))^(-1/2),   chord = 2 cos(delta/2) / (1/s_k + 1/s_{k+1}).
    Each half (half-angle h = delta/4 < pi/4) is covered by the quad of its circular sector of radius
    rho: vertices rho d(a), rho / cos(h) d(a + h), rho d(a + 2h) around the centre."""
    K = s.shape[0]
    verts = []
    for k in range(K):
        th_k = float(theta[k])
        th_n = float(theta[k + 1]) if k + 1 < K else float(theta[0]) + TWO_PI
        s_k = float(s[k])
        s_n = float(s[(k + 1) % K])
        dl = th_n - th_k
        sbar_mid = 1.0 / math.sqrt(0.5 * (1.0 / (s_k * s_k) + 1.0 / (s_n * s_n)))
        chord_mid = 2.0 * math.cos(0.5 * dl) / (1.0 / s_k + 1.0 / s_n)
        r_mid = max(sbar_mid, chord_mid)
        rho0 = c * max(s_k, r_mid)
        rho1 = c * max(s_n, r_mid)
        sec = 1.0 / math.cos(0.25 * dl)
        a1 = th_k + 0.5 * dl
        m0 = th_k + 0.25 * dl
        m1 = th_k + 0.75 * dl
        verts.append((rho0 * math.cos(th_k), rho0 * math.sin(th_k)))
        verts.append((rho0 * sec * math.cos(m0), rho0 * sec * math.sin(m0)))
        verts.append((rho0 * math.cos(a1), rho0 * math.sin(a1)))
        verts.append((rho1 * math.cos(a1), rho1 * math.sin(a1)))
        verts.append((rho1 * sec * math.cos(m1), rho1 * sec * math.sin(m1)))
        verts.append((rho1 * math.cos(th_n), rho1 * math.sin(th_n)))
    return np.array(verts)


def paper_polygon(s: np.ndarray, theta: np.ndarray, o: float, tau: float) -> np.ndarray:
    """The polygon of Sec. 4.4 as printed: endpoints at s_k * sqrt(-log Psi^{-1}(e^{-9}/o)).
    Not conservative (the L2 contours bulge past the chords)."""
    y = math.exp(-9.0) / o
    g = _psi_inv_scalar(min(y, 1.0), tau)
    ml = -math.log(g)
    fct = math.sqrt(ml if ml > 0.0 else 0.0)
    out = []
    for k in range(len(s)):
        sc = float(s[k]) * fct
        out.append((sc * math.cos(float(theta[k])), sc * math.sin(float(theta[k]))))
    return np.array(out)


def _clip_near(poly3: np.ndarray, near: float) -> np.ndarray:
    """Sutherland-Hodgman clip of a camera-space polygon to z >= near."""
    out = []
    nv = len(poly3)
    for i in range(nv):
        a = [float(v) for v in poly3[i]]
        b = [float(v) for v in poly3[(i + 1) % nv]]
        ain = a[2] >= near
        bin_ = b[2] >= near
        if ain:
            out.append(a)
        if ain != bin_:
            t = (near - a[2]) / (b[2] - a[2])
            out.append([a[k] + t * (b[k] - a[k]) for k in range(3)])
    return np.array(out).reshape(-1, 3)


def row_spans(poly2: np.ndarray, disk, W: int, H: int) -> Dict[int, Tuple[int, int]]:
    """Tile columns [i0, i1] per tile row touched by a screen polygon (and an optional square
    (cx, cy, r) around the projected centre for the low-pass support).  For a tile row the slab of
    pixel-centre heights [16j + 0.5, min(16j + 15.5, H - 0.5)] is intersected with every edge; the
    x-extent of the clipped edges (clamped to the pixel centres [0.5, W - 0.5]) picks the tiles whose
    centre columns it overlaps."""
    tx = (W + TILE - 1) // TILE
    ty = (H + TILE - 1) // TILE
    spans = {}
    nv = len(poly2)
    for j in range(ty):
        ya = TILE * j + 0.5
        yb = min(TILE * j + TILE - 0.5, H - 0.5)
        lo, hi = math.inf, -math.inf
        for e in range(nv):
            x0, y0 = poly2[e]
            x1, y1 = poly2[(e + 1) % nv]
            if max(y0, y1) < ya or min(y0, y1) > yb:
                continue
            if y0 == y1:
                xa, xb = x0, x1
            else:
                ta = (ya - y0) / (y1 - y0)
                tb = (yb - y0) / (y1 - y0)
                tlo = max(0.0, min(ta, tb))
                thi = min(1.0, max(ta, tb))
                xa = x0 + tlo * (x1 - x0)
                xb = x0 + thi * (x1 - x0)
            lo = min(lo, xa, xb)
            hi = max(hi, xa, xb)
        if disk is not None:
            dcx, dcy, r = disk
            if dcy + r >= ya and dcy - r <= yb:
                lo = min(lo, dcx - r)
                hi = max(hi, dcx + r)
        lo = max(lo, 0.5)
        hi = min(hi, W - 0.5)
        if lo > hi:
            continue
        i0 = max(math.ceil((lo - (TILE - 0.5)) / TILE), 0)
        i1 = min(math.floor((hi - 0.5) / TILE), tx - 1)
        if i0 <= i1:
            spans[j] = (i0, i1)
    return spans


def _rot_cols(q) -> List[List[float]]:
    """R(q) (row-major) for a quaternion (w, x, y, z), products and sums in the order written."""
    w, x, y, z = (float(a) for a in q)
    nrm = math.sqrt(((w * w + x * x) + y * y) + z * z)
    w, x, y, z = w / nrm, x / nrm, y / nrm, z / nrm
    return [[1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)],
            [2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)],
            [2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)]]


def _to_cam(Rc, tc, p):
    return [((Rc[i][0] * p[0] + Rc[i][1] * p[1]) + Rc[i][2] * p[2]) + tc[i] for i in range(3)]


def primitive_valid(scene, j: int) -> bool:
    """Parameter validity (R19 reading: invalid primitives are culled): finite centre and rotation,
    s_k > 0, angles in [0, 2*pi) with every gap (wrap included) in (0, pi), o in (0, 1],
    tau in (-1, 1), eta in [0, 1]."""
    f = lambda a: float(np.float32(a))
    mu = [f(scene.mu[i, j]) for i in range(3)]
    q = [f(scene.q[i, j]) for i in range(4)]
    if not all(math.isfinite(a) for a in mu + q):
        return False
    if not (((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3] > 0.0):
        return False
    K = scene.K
    s = [f(scene.scale[k, j]) for k in range(K)]
    th = [f(scene.theta[k, j]) for k in range(K)]
    if not all(math.isfinite(a) and a > 0.0 for a in s):
        return False
    if not all(0.0 <= a < TWO_PI for a in th):
        return False
    for k in range(K):
        nxt = th[k + 1] if k + 1 < K else th[0] + TWO_PI
        gap = nxt - th[k]
        if not (0.0 < gap < math.pi):
            return False
    o, tau, eta = f(scene.opacity[j]), f(scene.tau[j]), f(scene.eta[j])
    return 0.0 < o <= 1.0 and -1.0 < tau < 1.0 and 0.0 <= eta <= 1.0


def _psi_inv_scalar(y: float, tau: float) -> float:
    if y < (1.0 - tau) / 4.0:
        return y * (1.0 + tau) / (1.0 - tau)
    if y < (3.0 + tau) / 4.0:
        return (y * (1.0 - tau) + tau) / (1.0 + tau)
    return (y * (1.0 + tau) - 2.0 * tau) / (1.0 - tau)


def primitive_tiles(scene, camera, opts: Opts, j: int) -> List[int]:
    """Tile ids (row-major, tile_x fastest) that primitive j is binned to (Sec. 4.4 Kernel Culling,
    with the conservative polygon of ``support_polygon``).  float64, operations in written order."""
    W, H = camera.width, camera.height
    tx = (W + TILE - 1) // TILE
    if not primitive_valid(scene, j):
        return []
    sup = support_screen(scene, camera, opts, j)
    if sup is None:
        return []
    if opts.cull_mode == 2:
        return list(range(tx * ((H + TILE - 1) // TILE)))
    scr, disk = sup
    spans = row_spans(scr, disk, W, H)
    out = []
    for row in sorted(spans):
        i0, i1 = spans[row]
        out.extend(row * tx + i for i in range(i0, i1 + 1))
    return out


def support_screen(scene, camera, opts: Opts, j: int):
    """Projected support of primitive j: the near-clipped support polygon in pixel coordinates (P, 2)
    and, with the low-pass filter, the square (centre x, centre y, half-width) of the low-pass term.
    None when the centre is at or behind the near plane or the opacity is below alpha_min; with
    cull_mode 2, (None, None).  float64, operations in written order."""
    f = lambda a: float(np.float32(a))
    Rc = [[f(camera.R[i][k]) for k in range(3)] for i in range(3)]
    tc = [f(camera.t[i]) for i in range(3)]
    fx, fy, cx, cy = f(camera.fx), f(camera.fy), f(camera.cx), f(camera.cy)
    mu = [f(scene.mu[i, j]) for i in range(3)]
    mc = _to_cam(Rc, tc, mu)
    o, tau = f(scene.opacity[j]), f(scene.tau[j])
    if not mc[2] > opts.near or o < opts.alpha_min:
        return None
    if opts.cull_mode == 2:
        return None, None
    R = _rot_cols([scene.q[i, j] for i in range(4)])
    tu = [R[0][0], R[1][0], R[2][0]]
    tv = [R[0][1], R[1][1], R[2][1]]
    s = np.array([f(scene.scale[k, j]) for k in range(scene.K)])
    th = np.array([f(scene.theta[k, j]) for k in range(scene.K)])
    if opts.cull_mode == 1:
        poly = paper_polygon(s, th, o, tau)
    else:
        c = math.sqrt(-2.0 * math.log(_psi_inv_scalar(opts.alpha_min / o, tau)))
        poly = support_polygon(s, th, c)
    camp = []
    for x, y in poly:
        x, y = float(x), float(y)
        wpt = [(mu[i] + x * tu[i]) + y * tv[i] for i in range(3)]
        camp.append(_to_cam(Rc, tc, wpt))
    camp = _clip_near(np.array(camp), opts.near)
    scr = np.array([[(fx * p[0]) / p[2] + cx, (fy * p[1]) / p[2] + cy] for p in camp]).reshape(-1, 2)
    disk = None
    if opts.lowpass_sl > 0:
        r = opts.lowpass_sl * math.sqrt(2.0 * math.log(max(o / opts.alpha_min, 1.0)))
        disk = ((fx * mc[0]) / mc[2] + cx, (fy * mc[1]) / mc[2] + cy, r)
    return scr, disk


def tile_lists(scene, camera, opts: Opts, prim_ids: Optional[Sequence[int]] = None):
    """Reference binning: for every tile, the primitives binned to it ordered by (pre-sort key, index),
    the key being the centre depth or, with ``opts.key_mode``, the per-tile key.  Returns (tiles dict
    -> list of (key, j)), per-primitive tile lists, and the centre-depth keys (uint32)."""
    ids = range(scene.n) if prim_ids is None else prim_ids
    key = centre_depth_f32(scene.mu, camera).view(np.uint32)
    per_prim = {}
    tiles: Dict[int, List[Tuple[int, int]]] = {}
    for j in ids:
        tl = primitive_tiles(scene, camera, opts, int(j))
        per_prim[int(j)] = tl
        kp = key_plane(scene, camera, opts, int(j)) if (opts.key_mode != 0 and tl) else None
        for t in tl:
            k = int(key[j]) if kp is None else tile_key(kp, camera, opts, t)
            tiles.setdefault(t, []).append((k, int(j)))
    for t in tiles:
        tiles[t].sort()
    return tiles, per_prim, key


# ---------------------------------------------------------------------------------------------
# Pre-sort key variants and the sorting-accuracy measures (supplement, cache-sorting evaluation:
# tile-kernel pairs pre-sorted by the nearest distance between kernel and tile, or by the most
# centric point, before the per-pixel cache; accuracy, Kendall's tau and MAE of the depths composited
# front to back).  Readings: the distance is the view depth; "most centric" is the depth where the
# ray through the centre of the rectangle below meets the kernel's plane; "nearest" is
# the smallest such depth over the rectangle's four corner rays, which bounds the plane's depth over
# the whole rectangle from below because 1/depth is affine in the pixel coordinates.  Both are held
# to the depth range of the kernel's support disc (radius sqrt(2) c max_k s_k, which contains the
# support polygon).  Every value is float64 in the order written and rounded to float32 once, so the
# keys are reproducible bit for bit.  The rectangle is the tile's pixel-centre rectangle cut to the
# pixel box of the kernel's projected support (conservative polygon and low-pass square), so that
# both keys look at the part of the tile the kernel can cover.

KEY_CENTRE, KEY_CENTRIC, KEY_NEAREST = 0, 1, 2


@dataclasses.dataclass
class KeyPlane:
    a: Tuple[float, float, float]   # camera-frame plane normal t_u^c x t_v^c (not normalised)
    dN: float                       # a . mu_c
    zc: float                       # view depth of the centre
    zlo: float                      # depth range of the support disc, zlo >= near
    zhi: float
    box: Optional[Tuple[float, float, float, float]]   # pixel box (x0, x1, y0, y1) of the projected support


def key_plane(scene, camera, opts: Opts, j: int) -> KeyPlane:
    """Camera-frame plane and support depth range of DRK j for the per-tile keys."""
    f = lambda a: float(np.float32(a))
    Rc = [[f(camera.R[i][k]) for k in range(3)] for i in range(3)]
    tc = [f(camera.t[i]) for i in range(3)]
    mu = [f(scene.mu[i, j]) for i in range(3)]
    mc = _to_cam(Rc, tc, mu)
    R = _rot_cols([scene.q[i, j] for i in range(4)])
    tu = [R[0][0], R[1][0], R[2][0]]
    tv = [R[0][1], R[1][1], R[2][1]]
    tuc = [(Rc[i][0] * tu[0] + Rc[i][1] * tu[1]) + Rc[i][2] * tu[2] for i in range(3)]
    tvc = [(Rc[i][0] * tv[0] + Rc[i][1] * tv[1]) + Rc[i][2] * tv[2] for i in range(3)]
    a = (tuc[1] * tvc[2] - tuc[2] * tvc[1], tuc[2] * tvc[0] - tuc[0] * tvc[2], tuc[0] * tvc[1] - tuc[1] * tvc[0])
    dN = (a[0] * mc[0] + a[1] * mc[1]) + a[2] * mc[2]
    o, tau = f(scene.opacity[j]), f(scene.tau[j])
    c = math.sqrt(-2.0 * math.log(_psi_inv_scalar(opts.alpha_min / o, tau)))
    smax = max(f(scene.scale[k, j]) for k in range(scene.K))
    zr = (math.sqrt(2.0) * (c * smax)) * math.sqrt(tuc[2] * tuc[2] + tvc[2] * tvc[2])
    box = None
    if opts.cull_mode == 0:
        scr, disk = support_screen(scene, camera, opts, j)
        xs, ys = list(scr[:, 0]), list(scr[:, 1])
        if disk is not None:
            xs += [disk[0] - disk[2], disk[0] + disk[2]]
            ys += [disk[1] - disk[2], disk[1] + disk[2]]
        box = (min(xs), max(xs), min(ys), max(ys))
    return KeyPlane(a, dN, mc[2], max(mc[2] - zr, opts.near), mc[2] + zr, box)


def plane_depth(kp: KeyPlane, camera, opts: Opts, x: float, y: float) -> Optional[float]:
    """View depth where the ray through pixel point (x, y) meets the plane, or None when it meets it
    at or behind the near plane (or not at all)."""
    f = lambda a: float(np.float32(a))
    fx, fy, cx, cy = f(camera.fx), f(camera.fy), f(camera.cx), f(camera.cy)
    wd = (kp.a[0] * ((x - cx) / fx) + kp.a[1] * ((y - cy) / fy)) + kp.a[2]
    if wd == 0.0:
        return None
    z = kp.dN / wd
    return z if (z > opts.near and z < math.inf) else None


def tile_rect(camera, tile: int) -> Tuple[float, float, float, float]:
    """Pixel-centre rectangle (xa, xb, ya, yb) of a tile, cut at the image border."""
    tx = (camera.width + TILE - 1) // TILE
    x0, y0 = TILE * (tile % tx), TILE * (tile // tx)
    return (x0 + 0.5, min(x0 + TILE - 0.5, camera.width - 0.5), y0 + 0.5, min(y0 + TILE - 0.5, camera.height - 0.5))


def key_rect(kp: KeyPlane, camera, tile: int) -> Tuple[float, float, float, float]:
    """The part of a tile's pixel-centre rectangle that the kernel's projected support box covers
    (the whole rectangle when they do not overlap or no box is known)."""
    xa, xb, ya, yb = tile_rect(camera, tile)
    if kp.box is None:
        return xa, xb, ya, yb
    x0, x1, y0, y1 = max(xa, kp.box[0]), min(xb, kp.box[1]), max(ya, kp.box[2]), min(yb, kp.box[3])
    if x0 > x1 or y0 > y1:
        return xa, xb, ya, yb
    return x0, x1, y0, y1


def tile_key_value(kp: KeyPlane, camera, opts: Opts, tile: int, mode: int) -> float:
    """Per-tile pre-sort key (float64, before rounding) of the kernel with plane ``kp``."""
    xa, xb, ya, yb = key_rect(kp, camera, tile)
    if mode == KEY_CENTRIC:
        z = plane_depth(kp, camera, opts, 0.5 * (xa + xb), 0.5 * (ya + yb))
        z = kp.zc if z is None else z
    elif mode == KEY_NEAREST:
        zs = [d for d in (plane_depth(kp, camera, opts, x, y) for x, y in ((xa, ya), (xb, ya), (xa, yb), (xb, yb)))
              if d is not None]
        z = min(zs) if zs else kp.zlo
    else:
        raise ValueError(mode)
    return min(max(z, kp.zlo), kp.zhi)


def tile_key(kp: KeyPlane, camera, opts: Opts, tile: int) -> int:
    """uint32 bits of the float32 per-tile key (opts.key_mode 1 or 2); positive, so the bits sort
    like the values."""
    return int(np.float32(tile_key_value(kp, camera, opts, tile, opts.key_mode)).view(np.uint32))


def arrival_keys(scene, camera, opts: Opts, px: np.ndarray, py: np.ndarray):
    """Callable (pixel slot p, primitive j) -> uint32 pre-sort key that orders pixel p's arrivals."""
    if opts.key_mode == KEY_CENTRE:
        key = centre_depth_f32(scene.mu, camera).view(np.uint32)
        return lambda p, j: int(key[j])
    tx = (camera.width + TILE - 1) // TILE
    planes: Dict[int, KeyPlane] = {}
    memo: Dict[Tuple[int, int], int] = {}

    def akey(p, j):
        t = (int(py[p]) // TILE) * tx + int(px[p]) // TILE
        k = memo.get((t, j))
        if k is None:
            if j not in planes:
                planes[j] = key_plane(scene, camera, opts, j)
            k = memo[(t, j)] = tile_key(planes[j], camera, opts, t)
        return k
    return akey


def sort_metrics(seqs: Sequence[Sequence[float]], cap: Optional[int] = None) -> Dict[str, float]:
    """Disorder of front-to-back composited depth sequences (one per pixel, first ``cap`` entries):
    accuracy = share of positions holding the depth that the sorted sequence holds there;
    Kendall's tau = per-pixel (concordant - discordant) / (m (m - 1) / 2) between composite order and
    depth (ties count as neither), averaged over pixels with m >= 2;
    MAE = mean |depth at a position - sorted depth at that position|."""
    n_el = n_ok = 0
    err = 0.0
    taus = []
    for seq in seqs:
        z = np.asarray(list(seq)[:cap] if cap else list(seq), dtype=np.float64)
        m = z.size
        if m == 0:
            continue
        zs = np.sort(z, kind="stable")
        n_el += m
        n_ok += int((z == zs).sum())
        err += float(np.abs(z - zs).sum())
        if m >= 2:
            later = np.triu(np.ones((m, m), bool), 1)
            d = z[None, :] - z[:, None]          # d[i, k] = z_k - z_i
            cd = int((d[later] > 0).sum()) - int((d[later] < 0).sum())
            taus.append(cd / (m * (m - 1) / 2))
    return dict(accuracy=n_ok / n_el if n_el else float("nan"),
                kendall_tau=float(np.mean(taus)) if taus else float("nan"),
                mae=err / n_el if n_el else float("nan"), n=n_el, pixels=len(taus))


# ---------------------------------------------------------------------------------------------
# Mesh to DRK (the section "Converting Mesh to DRK" and its supplement): one DRK per planar convex face,
# with the basis endpoints at the face's vertices.  Readings: the centre is the mean of the
# vertices; the plane frame has t_u toward the first vertex and the normal of the face's winding
# (sum of the cross products of consecutive centred vertices); theta_k are the vertex directions in
# the listed order (theta_0 = 0); eta = 1, so the L1 level sets (Eq. L1) are the face polygon
# itself, and s_k = d_k / sqrt(2 ln 2) puts the vertices on the level E = 2 ln 2, where g = 1/2 and
# Psi(g) = 1/2 for every tau: the half-opacity contour is the face outline, and tau sets how sharp
# it is.  A face with m < K vertices gets K - m extra endpoints on its edges: edge i (from vertex i
# to vertex i+1) takes floor((K - m) / m) of them, plus one when i < (K - m) mod m, evenly spaced
# along it; endpoints on the edges leave the L1 polygon unchanged.

MESH_LEVEL = math.sqrt(2.0 * math.log(2.0))


def _quat_from_frame(tu, tv, n):
    """(w, x, y, z) of the rotation whose columns are t_u, t_v, n (Shepperd's method)."""
    R = [[tu[0], tv[0], n[0]], [tu[1], tv[1], n[1]], [tu[2], tv[2], n[2]]]
    t = R[0][0] + R[1][1] + R[2][2]
    if t > 0.0:
        r = math.sqrt(1.0 + t)
        return (0.5 * r, (R[2][1] - R[1][2]) / (2.0 * r), (R[0][2] - R[2][0]) / (2.0 * r), (R[1][0] - R[0][1]) / (2.0 * r))
    i = max(range(3), key=lambda k: R[k][k])
    j, k = (i + 1) % 3, (i + 2) % 3
    r = math.sqrt(1.0 + R[i][i] - R[j][j] - R[k][k])
    q = [0.0, 0.0, 0.0, 0.0]
    q[0] = (R[k][j] - R[j][k]) / (2.0 * r)
    q[1 + i] = 0.5 * r
    q[1 + j] = (R[j][i] + R[i][j]) / (2.0 * r)
    q[1 + k] = (R[k][i] + R[i][k]) / (2.0 * r)
    return tuple(q)


def mesh_face_drk(P: np.ndarray, K: int):
    """One face (m, 3) -> (mu, (t_u, t_v, n), theta[K], s[K]) in float64, or None when the face is
    degenerate, not convex, or wound the other way round its own normal."""
    P = np.asarray(P, np.float64)
    m = len(P)
    if m < 3 or m > K:
        return None
    mu = P.mean(axis=0)
    D = P - mu
    a = np.zeros(3)
    for i in range(m):
        a += np.cross(D[i], D[(i + 1) % m])
    na = float(np.linalg.norm(a))
    d0 = float(np.linalg.norm(D[0]))
    if not (na > 0.0 and d0 > 0.0):
        return None
    n = a / na
    tu = D[0] / d0
    tv = np.cross(n, tu)
    x = [float(D[i] @ tu) for i in range(m)]
    y = [float(D[i] @ tv) for i in range(m)]
    ang = [0.0] + [math.atan2(y[i], x[i]) % TWO_PI for i in range(1, m)]
    # extra endpoints on the edges, round robin from edge 0
    extra = [(K - m) // m + (1 if i < (K - m) % m else 0) for i in range(m)]
    xs, ys, th = [], [], []
    for i in range(m):
        xa, ya, xb, yb = x[i], y[i], x[(i + 1) % m], y[(i + 1) % m]
        xs.append(xa)
        ys.append(ya)
        th.append(ang[i])
        for c in range(1, extra[i] + 1):
            f = c / (extra[i] + 1)
            px, py = xa + f * (xb - xa), ya + f * (yb - ya)
            xs.append(px)
            ys.append(py)
            th.append(math.atan2(py, px) % TWO_PI)
    for k in range(1, K):
        gap = th[k] - th[k - 1]
        if not (0.0 < gap < math.pi):
            return None
    if not (0.0 < th[0] + TWO_PI - th[K - 1] < math.pi):
        return None
    s = [math.hypot(xs[k], ys[k]) / MESH_LEVEL for k in range(K)]
    return mu, (tu, tv, n), th, s


def mesh_to_drk(vertices: np.ndarray, faces: np.ndarray, colors: np.ndarray, K: int, tau: float = 0.95,
                opacity: float = 0.99):
    """Converts a polygon mesh (vertices (nv, 3); faces (nf, m) vertex indices, -1 padding; RGB per
    face (nf, 3)) to a DRK scene with K bases (float32 SoA).  Vertices are taken in float32 (as the
    ABI carries them) and promoted exactly.  Faces that cannot be converted get opacity 0 (culled by
    the renderer)."""
    from drk_synth import Scene
    V = np.asarray(vertices, np.float32).astype(np.float64)
    F = np.asarray(faces)
    nf = F.shape[0]
    mu = np.zeros((3, nf))
    q = np.zeros((4, nf))
    q[0] = 1.0
    sc = np.ones((K, nf))
    th = np.tile((np.arange(K) * (TWO_PI / K))[:, None], (1, nf))
    op = np.zeros(nf)
    for f in range(nf):
        idx = [int(i) for i in F[f] if i >= 0]
        r = mesh_face_drk(V[idx], K)
        if r is None:
            continue
        m_, (tu, tv, n), t_, s_ = r
        mu[:, f] = m_
        q[:, f] = _quat_from_frame(tu, tv, n)
        sc[:, f] = s_
        th[:, f] = t_
        op[f] = opacity
    th32 = np.minimum(th.astype(np.float32), np.nextafter(np.float32(TWO_PI), np.float32(0)))
    return Scene(mu.astype(np.float32), q.astype(np.float32), sc.astype(np.float32), th32,
                 np.ones(nf, np.float32), np.full(nf, tau, np.float32), op.astype(np.float32),
                 np.ascontiguousarray(np.asarray(colors, np.float32).T), -1)


# ---------------------------------------------------------------------------------------------
# Parametrization and the optimizer step (supplement S4, Parametrization and Model Training).
# Raw (unconstrained) parameters map to the renderer's: o = sigmoid, s_k = exp, q normalised,
# tau = -0.1 + 1.09 sigmoid (the range (-0.1, 0.99)), eta = sigmoid, colour and centre unchanged.
# Angles (reading): the K sector gaps are proportional to a_k = sigmoid(raw_k) + 1/(K - 2) and sum to
# 2 pi; theta_k is their cumulative sum before k (theta_0 = 0; q carries the kernel's rotation).
# Since a_k lies in (1/(K-2), 1 + 1/(K-2)), every gap is below (1 + 1/(K-2)) / (1 + 1/(K-2) +
# (K-1)/(K-2)) = 1/2 of the turn: the residual is what keeps the sectors under pi.

TAU_LO, TAU_SPAN = -0.1, 1.09


def activate(raw: Dict[str, torch.Tensor]) -> Dict[str, torch.Tensor]:
    """Raw parameters (float64 tensors, keys mu, q [N, 4], scale / theta [N, K], eta, tau,
    opacity [N], color) -> activated parameters, differentiably."""
    K = raw["theta"].shape[-1]
    a = torch.sigmoid(raw["theta"]) + 1.0 / (K - 2)
    gaps = TWO_PI * a / a.sum(-1, keepdim=True)
    theta = torch.cumsum(gaps, -1) - gaps
    return {"mu": raw["mu"], "q": raw["q"] / torch.linalg.vector_norm(raw["q"], dim=-1, keepdim=True),
            "scale": torch.exp(raw["scale"]), "theta": theta, "eta": torch.sigmoid(raw["eta"]),
            "tau": TAU_LO + TAU_SPAN * torch.sigmoid(raw["tau"]), "opacity": torch.sigmoid(raw["opacity"]),
            "color": raw["color"]}


def activate_vjp(raw: Dict[str, torch.Tensor], g_act: Dict[str, torch.Tensor]) -> Dict[str, torch.Tensor]:
    """Gradient with respect to the raw parameters of sum(g_act * activate(raw)) (float64 autograd)."""
    leaves = {k: v.detach().clone().requires_grad_(True) for k, v in raw.items()}
    act = activate(leaves)
    total = sum((act[k] * g_act[k]).sum() for k in act)
    total.backward()
    return {k: v.grad.detach() for k, v in leaves.items()}


def adam_step(p, m, v, g, lr, beta1, beta2, eps, step):
    """One Adam update (Kingma and Ba), bias-corrected, step >= 1; returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
