"""Python binding of libdrk: torch tensors in, torch tensors out.  Every step runs in the HIP
library; this module only builds the C structs, passes data pointers and the current HIP stream,
and applies the overflow-retry policy of the pair buffer."""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import DRK_OK, DRK_EOVERFLOW, check, lib

EXPORT = {"depth_keys": 0, "tile_counts": 1, "pair_tiles": 2, "pair_prims": 3, "ranges": 4, "emitted": 5,
          "consumed": 6, "contributors": 7, "hits": 8, "kernels": 9, "pair_keys": 10}
KEY_MODES = {"centre": 0, "centric": 1, "nearest": 2}


def _stream_handle(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


@dataclasses.dataclass
class DRKScene:
    """Scene arrays on the GPU, float32, SoA ([rows][n])."""
    mu: torch.Tensor
    q: torch.Tensor
    scale: torch.Tensor
    theta: torch.Tensor
    eta: torch.Tensor
    tau: torch.Tensor
    opacity: torch.Tensor
    color: torch.Tensor
    sh_degree: int = -1

    FIELDS = ("mu", "q", "scale", "theta", "eta", "tau", "opacity", "color")

    @property
    def n(self) -> int:
        return int(self.mu.shape[-1])

    @property
    def K(self) -> int:
        return int(self.scale.shape[0])

    @staticmethod
    def from_host(scene, device="cuda") -> "DRKScene":
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return DRKScene(t(scene.mu), t(scene.q), t(scene.scale), t(scene.theta), t(scene.eta), t(scene.tau),
                        t(scene.opacity), t(scene.color), int(scene.sh_degree))

    def tensors(self):
        return [getattr(self, f) for f in self.FIELDS]

    def c_struct(self) -> _lib.Scene:
        for f in self.FIELDS:
            a = getattr(self, f)
            if a.dtype != torch.float32 or not a.is_contiguous() or not a.is_cuda:
                raise ValueError(f"scene.{f} must be a contiguous float32 CUDA tensor")
        s = _lib.Scene()
        s.n = self.n
        s.K = self.K
        s.color_mode = 0 if self.sh_degree < 0 else 1
        s.sh_degree = max(self.sh_degree, 0)
        for f in self.FIELDS:
            setattr(s, f, getattr(self, f).data_ptr())
        return s


def camera_struct(cam) -> _lib.Camera:
    c = _lib.Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, np.float32).reshape(9)
    t = np.asarray(cam.t, np.float32).reshape(3)
    bg = np.asarray(getattr(cam, "bg", np.zeros(3)), np.float32).reshape(3)
    c.R[:] = [float(x) for x in R]
    c.t[:] = [float(x) for x in t]
    c.bg[:] = [float(x) for x in bg]
    return c


def make_opts(alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4, near=0.2, lowpass_sl=math.sqrt(0.5),
              cache_len=8, cull_mode=0, validate=0, key_mode=0, launch_order=0, counters=0) -> _lib.Opts:
    """key_mode: 0 / "centre", 1 / "centric", 2 / "nearest" (pre-sort key of the tile lists);
    launch_order: 0 longest tile lists first, 1 row-major; counters: 1 = the forward also writes the
    per-pixel work counters (exports emitted, consumed, contributors, hits, kernels) (see drk_opts)."""
    o = _lib.Opts()
    o.alpha_min, o.alpha_max, o.T_min, o.near_plane, o.lowpass_sl = alpha_min, alpha_max, T_min, near, lowpass_sl
    o.cache_len, o.cull_mode, o.validate = cache_len, cull_mode, validate
    o.key_mode = KEY_MODES[key_mode] if isinstance(key_mode, str) else int(key_mode)
    o.launch_order = int(launch_order)
    o.counters = int(counters)
    return o


class Rasterizer:
    """Owns a libdrk workspace (device memory for up to max_views views of max_n primitives)."""

    def __init__(self, max_n: int, K: int, max_w: int, max_h: int, max_views: int = 1,
                 pair_capacity: int = 1 << 24, grow: bool = True):
        self.max_n, self.K, self.max_w, self.max_h, self.max_views = max_n, K, max_w, max_h, max_views
        self.pair_capacity = int(pair_capacity)
        self.grow = grow
        self._ws = C.c_void_p()
        self._create()
        self._cams: List = []
        self._scene: Optional[DRKScene] = None
        self._opts = None

    def _create(self):
        check(lib().drk_ws_create(self.max_n, self.K, self.max_views, self.max_w, self.max_h, self.pair_capacity,
                                  C.byref(self._ws)), "drk_ws_create")

    def close(self):
        if self._ws:
            lib().drk_ws_destroy(self._ws)
            self._ws = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def size_query(max_n, K, max_w, max_h, max_views=1, pair_capacity=1 << 24) -> int:
        b = C.c_size_t()
        check(lib().drk_ws_size_query(max_n, K, max_views, max_w, max_h, pair_capacity, C.byref(b)))
        return int(b.value)

    # -- the four steps ---------------------------------------------------------------------
    def preprocess(self, scene: DRKScene, cams: Sequence, opts=None):
        opts = opts if opts is not None else make_opts()
        arr = (_lib.Camera * len(cams))(*[camera_struct(c) for c in cams])
        self._cstruct = scene.c_struct()
        check(lib().drk_preprocess(self._ws, C.byref(self._cstruct), arr, len(cams), C.byref(opts),
                                   C.c_void_p(_stream_handle())), "drk_preprocess")
        self._cams, self._scene, self._opts = list(cams), scene, opts

    def bin_sort(self):
        check(lib().drk_bin_sort(self._ws, C.c_void_p(_stream_handle())), "drk_bin_sort")

    def render_fwd(self, rgb: Optional[torch.Tensor] = None, T: Optional[torch.Tensor] = None):
        npx = sum(int(c.width) * int(c.height) for c in self._cams)
        dev = self._scene.mu.device
        if rgb is None:
            rgb = torch.empty(3 * npx, dtype=torch.float32, device=dev)
        if T is None:
            T = torch.empty(npx, dtype=torch.float32, device=dev)
        check(lib().drk_render_fwd(self._ws, _ptr(rgb), _ptr(T), C.c_void_p(_stream_handle())), "drk_render_fwd")
        return rgb, T

    def render_trace(self, cap: int = 64):
        """Forward render that also records each pixel's composited contributions front to back.
        Returns rgb (flat), T (flat), trace_n [px], trace_idx [px][cap], trace_z [px][cap]."""
        npx = sum(int(c.width) * int(c.height) for c in self._cams)
        dev = self._scene.mu.device
        rgb = torch.empty(3 * npx, dtype=torch.float32, device=dev)
        T = torch.empty(npx, dtype=torch.float32, device=dev)
        tn = torch.empty(npx, dtype=torch.int32, device=dev)
        ti = torch.full((npx, cap), -1, dtype=torch.int32, device=dev)
        tz = torch.full((npx, cap), float("nan"), dtype=torch.float32, device=dev)
        check(lib().drk_render_trace(self._ws, _ptr(rgb), _ptr(T), int(cap), _ptr(tn), _ptr(ti), _ptr(tz),
                                     C.c_void_p(_stream_handle())), "drk_render_trace")
        return rgb, T, tn, ti, tz

    def render_depth_normal(self):
        """Forward render with the depth [px] and normal [3][px] channels (flat, views packed).
        Returns rgb, T, depth, normal."""
        npx = sum(int(c.width) * int(c.height) for c in self._cams)
        dev = self._scene.mu.device
        rgb = torch.empty(3 * npx, dtype=torch.float32, device=dev)
        T = torch.empty(npx, dtype=torch.float32, device=dev)
        depth = torch.empty(npx, dtype=torch.float32, device=dev)
        normal = torch.empty(3 * npx, dtype=torch.float32, device=dev)
        check(lib().drk_render_depth_normal(self._ws, _ptr(rgb), _ptr(T), _ptr(depth), _ptr(normal),
                                            C.c_void_p(_stream_handle())), "drk_render_depth_normal")
        return rgb, T, depth, normal

    def render_bwd(self, rgb: torch.Tensor, dL_drgb: torch.Tensor) -> DRKScene:
        sc = self._scene
        g = DRKScene(*[torch.empty_like(t) for t in sc.tensors()], sh_degree=sc.sh_degree)
        gs = _lib.SceneGrad(*[t.data_ptr() for t in g.tensors()])
        check(lib().drk_render_bwd(self._ws, C.byref(self._cstruct), _ptr(rgb.contiguous()),
                                   _ptr(dL_drgb.contiguous()), C.byref(gs), C.c_void_p(_stream_handle())),
              "drk_render_bwd")
        return g

    def generation(self) -> int:
        """drk_preprocess calls made on this workspace (identifies the frame its lists belong to)."""
        g = C.c_uint64()
        check(lib().drk_ws_generation(self._ws, C.byref(g)), "drk_ws_generation")
        return int(g.value)

    def status(self):
        need = C.c_int64()
        code = lib().drk_ws_status(self._ws, C.c_void_p(_stream_handle()), C.byref(need))
        return code, int(need.value)

    def export(self, what: str, view: int = 0) -> torch.Tensor:
        cnt = C.c_int64()
        code = EXPORT[what]
        check(lib().drk_ws_export(self._ws, view, code, None, 0, C.byref(cnt), C.c_void_p(_stream_handle())))
        out = torch.empty(int(cnt.value), dtype=torch.int32, device=self._scene.mu.device)
        check(lib().drk_ws_export(self._ws, view, code, _ptr(out), out.numel() * 4, C.byref(cnt),
                                  C.c_void_p(_stream_handle())), "drk_ws_export")
        return out   # int32; unsigned exports are reinterpreted by the caller

    # -- convenience ------------------------------------------------------------------------
    def forward(self, scene: DRKScene, cams: Sequence, opts=None, check_overflow: bool = True):
        """preprocess -> bin_sort -> render_fwd.  Returns rgb (V, 3, H, W) and T (V, H, W) when all
        views share a size, else flat buffers.  On pair-buffer overflow the workspace is recreated
        with a larger capacity and the frame is redone (when ``grow``)."""
        while True:
            self.preprocess(scene, cams, opts)
            self.bin_sort()
            if check_overflow:
                code, need = self.status()
                if code == DRK_EOVERFLOW and self.grow:
                    self.close()
                    self.pair_capacity = int(need * 1.25) + 1024
                    self._create()
                    continue
                if code != DRK_OK:
                    check(code, "drk_bin_sort")
            break
        rgb, T = self.render_fwd()
        return self._shape(rgb, T)

    def _shape(self, rgb, T):
        sizes = {(int(c.width), int(c.height)) for c in self._cams}
        if len(sizes) == 1:
            (W, H), = sizes
            V = len(self._cams)
            return rgb.view(V, 3, H, W), T.view(V, H, W)
        return rgb, T


class DRKRenderFunction(torch.autograd.Function):
    """Differentiable DRK render through libdrk (forward: drk_render_fwd; backward: drk_render_bwd)."""

    @staticmethod
    def forward(ctx, ras: Rasterizer, cams, opts, sh_degree, mu, q, scale, theta, eta, tau, opacity, color):
        scene = DRKScene(mu.detach().contiguous(), q.detach().contiguous(), scale.detach().contiguous(),
                         theta.detach().contiguous(), eta.detach().contiguous(), tau.detach().contiguous(),
                         opacity.detach().contiguous(), color.detach().contiguous(), sh_degree)
        rgb, T = ras.forward(scene, cams, opts)
        ctx.ras = ras
        ctx.generation = ras.generation()
        ctx.scene = scene
        ctx.save_for_backward(rgb)
        ctx.mark_non_differentiable(T)
        return rgb, T

    @staticmethod
    def backward(ctx, g_rgb, g_T):
        rgb, = ctx.saved_tensors
        if ctx.ras.generation() != ctx.generation:
            raise RuntimeError("the rasterizer rendered another frame after this forward pass: its lists no "
                               "longer belong to this output (use one Rasterizer per pending backward)")
        g = ctx.ras.render_bwd(rgb.reshape(-1), g_rgb.contiguous().reshape(-1))
        return (None, None, None, None, *g.tensors())


def render(ras: Rasterizer, scene: DRKScene, cams, opts=None):
    """Differentiable render of the scene tensors (which may require grad)."""
    return DRKRenderFunction.apply(ras, cams, opts, scene.sh_degree, *scene.tensors())


def trace_metrics(trace_n: torch.Tensor, trace_z: torch.Tensor, cap: int) -> dict:
    """Sorting-accuracy measures of traces from ``Rasterizer.render_trace`` (cap <= 64), computed by
    drk_trace_metrics: accuracy, mean Kendall's tau, MAE of the composited depths against their
    sorted order, plus the counts they are taken over."""
    if trace_z.shape[-1] != cap:
        raise ValueError("trace_z must be [px][cap]")
    out = torch.empty(6, dtype=torch.float64, device=trace_n.device)
    check(lib().drk_trace_metrics(_ptr(trace_n.contiguous()), _ptr(trace_z.contiguous()), int(trace_n.numel()),
                                  int(cap), _ptr(out), C.c_void_p(_stream_handle(trace_n.device))), "drk_trace_metrics")
    n, ok, tau, npx2, err, trunc = out.cpu().tolist()
    return dict(accuracy=ok / n if n else float("nan"), kendall_tau=tau / npx2 if npx2 else float("nan"),
                mae=err / n if n else float("nan"), n=int(n), pixels=int(npx2), truncated=int(trunc))


def mesh_to_drk(vertices: torch.Tensor, faces: torch.Tensor, face_rgb: torch.Tensor, K: int, tau: float = 0.95,
                opacity: float = 0.99):
    """Converts a polygon mesh on the GPU to a DRK scene (drk_mesh_to_drk): vertices [3][nv] float32,
    faces [nf][m] int32 (-1 pads short faces), face_rgb [3][nf] float32, all CUDA tensors.
    Returns (DRKScene with RGB colour, number of rejected faces)."""
    for name, t, dt in (("vertices", vertices, torch.float32), ("faces", faces, torch.int32),
                        ("face_rgb", face_rgb, torch.float32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dt} CUDA tensor")
    nv, (nf, m) = int(vertices.shape[1]), faces.shape
    dev = vertices.device
    f32 = lambda *shape: torch.empty(*shape, dtype=torch.float32, device=dev)
    sc = DRKScene(f32(3, nf), f32(4, nf), f32(K, nf), f32(K, nf), f32(nf), f32(nf), f32(nf), f32(3, nf), -1)
    out = _lib.SceneOut(*[t.data_ptr() for t in sc.tensors()])
    rej = torch.zeros(1, dtype=torch.int32, device=dev)
    check(lib().drk_mesh_to_drk(_ptr(vertices), nv, _ptr(faces), int(nf), int(m), _ptr(face_rgb), int(K),
                                float(tau), float(opacity), C.byref(out), _ptr(rej), C.c_void_p(_stream_handle(dev))),
          "drk_mesh_to_drk")
    return sc, int(rej.item())


def _scene_like(sc: DRKScene) -> DRKScene:
    return DRKScene(*[torch.empty_like(t) for t in sc.tensors()], sh_degree=sc.sh_degree)


def activate(raw: DRKScene) -> DRKScene:
    """Raw, unconstrained parameters -> the renderer's parameters (drk_activate; supplement S4)."""
    out = _scene_like(raw)
    o = _lib.SceneOut(*[t.data_ptr() for t in out.tensors()])
    cs = raw.c_struct()
    check(lib().drk_activate(C.byref(cs), C.byref(o), C.c_void_p(_stream_handle(raw.mu.device))), "drk_activate")
    return out


def activate_bwd(raw: DRKScene, g_act: DRKScene) -> DRKScene:
    """dL/d(raw) from dL/d(activated) (drk_activate_bwd)."""
    out = _scene_like(raw)
    o = _lib.SceneOut(*[t.data_ptr() for t in out.tensors()])
    g = _lib.SceneGrad(*[t.contiguous().data_ptr() for t in g_act.tensors()])
    cs = raw.c_struct()
    check(lib().drk_activate_bwd(C.byref(cs), C.byref(g), C.byref(o), C.c_void_p(_stream_handle(raw.mu.device))),
          "drk_activate_bwd")
    return out


def adam_step(param: torch.Tensor, m: torch.Tensor, v: torch.Tensor, grad: torch.Tensor, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, step: int = 1) -> None:
    """In-place bias-corrected Adam on contiguous float32 CUDA tensors of equal size (drk_adam_step)."""
    for t in (param, m, v, grad):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != param.numel():
            raise ValueError("adam_step needs contiguous float32 CUDA tensors of one size")
    check(lib().drk_adam_step(_ptr(param), _ptr(m), _ptr(v), _ptr(grad), int(param.numel()), float(lr), float(beta1),
                              float(beta2), float(eps), int(step), C.c_void_p(_stream_handle(param.device))),
          "drk_adam_step")
