"""Python binding of libdrk's serving loop (drk_serve_*): argument marshalling only."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import torch

from . import _lib
from ._lib import DRK_EAGAIN, check, lib
from .rasterizer import DRKScene, camera_struct, make_opts


class Server:
    """Continuous-batching render server on the current GPU."""

    def __init__(self, hbm_budget_bytes: int = 0, max_inflight: int = 4, queue_capacity: int = 4096,
                 use_graphs: bool = True, opts=None, initial_pairs: int = 0):
        cfg = _lib.ServeCfg()
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.max_inflight = int(max_inflight)
        cfg.queue_capacity = int(queue_capacity)
        cfg.use_graphs = 1 if use_graphs else 0
        cfg.initial_pairs = int(initial_pairs)
        cfg.opts = opts if opts is not None else make_opts()
        self._srv = C.c_void_p()
        check(lib().drk_serve_create(C.byref(cfg), C.byref(self._srv)), "drk_serve_create")

    def close(self):
        if self._srv:
            lib().drk_serve_destroy(self._srv)
            self._srv = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_scene(self, scene: DRKScene) -> int:
        sid = C.c_int32()
        cs = scene.c_struct()
        check(lib().drk_serve_add_scene(self._srv, C.byref(cs), C.byref(sid)), "drk_serve_add_scene")
        return int(sid.value)

    def submit(self, scene_id: int, cam, out: torch.Tensor) -> int:
        """Returns the request id; raises DrkError (DRK_EAGAIN when the queue is full)."""
        c = camera_struct(cam)
        rid = C.c_uint64()
        check(lib().drk_serve_submit(self._srv, int(scene_id), C.byref(c), C.c_void_p(out.data_ptr()), C.byref(rid)),
              "drk_serve_submit")
        return int(rid.value)

    def try_submit(self, scene_id: int, cam, out: torch.Tensor):
        c = camera_struct(cam)
        rid = C.c_uint64()
        code = lib().drk_serve_submit(self._srv, int(scene_id), C.byref(c), C.c_void_p(out.data_ptr()), C.byref(rid))
        return code, int(rid.value)

    def poll(self, request_id: int, wait_us: int = 0) -> Optional[dict]:
        """Stats dict when the request is done (it is then forgotten), None while pending."""
        st = _lib.ReqStats()
        code = lib().drk_serve_poll(self._srv, C.c_uint64(request_id), int(wait_us), C.byref(st))
        if code == DRK_EAGAIN:
            return None
        check(code, "drk_serve_poll")
        return {"submit_us": st.submit_us, "start_us": st.start_us, "done_us": st.done_us, "pairs": st.pairs,
                "status": st.status, "width": st.width, "height": st.height}

    def wait(self, request_id: int) -> dict:
        while True:
            r = self.poll(request_id, wait_us=100_000)
            if r is not None:
                return r
