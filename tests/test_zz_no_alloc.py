"""The forward entry point that allocates nothing (drk_render_fwd_noalloc): its intermediates live in
the library's fixed device array.  Two calls in a row, the second with a smaller scene and image,
each equal to the workspace path (drk_preprocess -> drk_bin_sort -> drk_render_fwd) on the same
input, and both within the oracle's tolerance; a scene too large for the array is refused."""
import ctypes as C

import numpy as np
import pytest
import torch

from drk_synth import camera_lookat, config_c1, config_c2, scene_uniform_box
from oracle import drk_oracle as O
from tests._gpu_util import IMG_TOL, compare_image, gpu_opts, log, need_gpu, oracle_opts

pytestmark = pytest.mark.gpu


def _noalloc(ds, cam, opts):
    from paper_2412_11752_amd import camera_struct
    from paper_2412_11752_amd._lib import lib
    rgb = torch.empty(3 * cam.width * cam.height, device="cuda")
    T = torch.empty(cam.width * cam.height, device="cuda")
    cs = ds.c_struct()
    cc = camera_struct(cam)
    code = lib().drk_render_fwd_noalloc(C.byref(cs), C.byref(cc), C.byref(opts), C.c_void_p(rgb.data_ptr()),
                                        C.c_void_p(T.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return code, rgb, T


def _workspace(ds, cam, opts):
    from paper_2412_11752_amd import Rasterizer
    ras = Rasterizer(ds.n, ds.K, cam.width, cam.height, pair_capacity=1 << 22)
    rgb, T = ras.forward(ds, [cam], opts)
    torch.cuda.synchronize()
    ras.close()
    return rgb.reshape(-1), T.reshape(-1)


def test_noalloc_matches_the_workspace_path_twice():
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    from paper_2412_11752_amd._lib import DRK_OK
    big, big_cam = config_c2(n=20_000)
    big_cam = camera_lookat((0.4, -3.2, 1.0), (0, 0, 0), (0, 0, 1), 331, 257, 60.0, bg=(0.1, 0.2, 0.3))
    small, small_cam = config_c1()
    opts = gpu_opts()
    for label, scene, cam in (("20k DRKs SH3 331x257", big, big_cam), ("256 DRKs RGB 64x64", small, small_cam)):
        ds = DRKScene.from_host(scene)
        code, rgb, T = _noalloc(ds, cam, opts)
        torch.cuda.synchronize()
        assert code == DRK_OK, label
        ref_rgb, ref_T = _workspace(ds, cam, opts)
        assert torch.equal(rgb, ref_rgb), label
        assert torch.equal(T, ref_T), label
        orc = O.render_image(scene, cam, oracle_opts())
        worst, nk, _, _ = compare_image(rgb.view(3, cam.height, cam.width).cpu().numpy(), orc, cam.height, cam.width)
        log(f"no-alloc {label}: bitwise equal to the workspace path, max err {worst:.2e} vs the oracle, knife {nk}")
        assert worst <= IMG_TOL, label


def test_noalloc_refuses_what_does_not_fit():
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    from paper_2412_11752_amd._lib import DRK_EINVAL, DRK_ENOMEM, lib
    scene = scene_uniform_box(3, 400_000, K=16)
    cam = camera_lookat((0, 0, -3.0), (0, 0, 0), (0, 1, 0), 1920, 1080, 60.0)
    ds = DRKScene.from_host(scene)
    code, _, _ = _noalloc(ds, cam, gpu_opts())
    assert code == DRK_ENOMEM
    msg = lib().drk_last_error().decode()
    log(f"refused: {msg}")
    assert "fixed device array" in msg
    small, small_cam = config_c1()
    code, _, _ = _noalloc(DRKScene.from_host(small), small_cam, gpu_opts(counters=1))
    assert code == DRK_EINVAL
