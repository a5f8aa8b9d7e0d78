"""libdrk's C ABI without a GPU: the library loads, exports every symbol include/drk.h declares,
and rejects invalid arguments on the host before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2412_11752_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "drk.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(drk_[a-z_]+)\s*\(", text)))


def test_header_declares_the_path():
    names = _declared()
    for n in ("drk_preprocess", "drk_bin_sort", "drk_render_fwd", "drk_render_bwd", "drk_serve_submit",
              "drk_serve_poll"):
        assert n in names
    assert set(names) == set(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for n in _declared():
        assert hasattr(L, n), n


def test_defaults_and_version():
    L = _lib.lib()
    o = L.drk_opts_default()
    assert o.alpha_min == pytest.approx(1 / 255) and o.alpha_max == pytest.approx(0.99)
    assert o.T_min == pytest.approx(1e-4) and o.near_plane == pytest.approx(0.2)
    assert o.lowpass_sl == pytest.approx(2 ** -0.5) and o.cache_len == 8 and o.cull_mode == 0
    assert b"gfx950" in L.drk_version()


def test_host_side_argument_errors():
    L = _lib.lib()
    ws = C.c_void_p()
    assert L.drk_ws_create(100, 2, 1, 64, 64, 1000, C.byref(ws)) == _lib.DRK_EINVAL      # K < 3
    assert b"K must be" in L.drk_last_error()
    assert L.drk_ws_create(100, 8, 0, 64, 64, 1000, C.byref(ws)) == _lib.DRK_EINVAL      # no views
    assert L.drk_ws_create(100, 8, 1, 64, 99999, 1000, C.byref(ws)) == _lib.DRK_EINVAL   # too tall
    assert L.drk_ws_create(100, 8, 1, 64, 64, 0, C.byref(ws)) == _lib.DRK_EINVAL         # no pairs
    assert L.drk_preprocess(None, None, None, 1, None, None) == _lib.DRK_EINVAL
    assert L.drk_bin_sort(None, None) == _lib.DRK_EINVAL
    assert L.drk_render_fwd(None, None, None, None) == _lib.DRK_EINVAL


def test_workspace_size_query():
    b8 = C.c_size_t()
    b16 = C.c_size_t()
    L = _lib.lib()
    assert L.drk_ws_size_query(1_000_000, 8, 1, 1920, 1080, 1 << 26, C.byref(b8)) == 0
    assert L.drk_ws_size_query(1_000_000, 16, 1, 1920, 1080, 1 << 26, C.byref(b16)) == 0
    assert b16.value > b8.value > 1_000_000 * 92 * 4


def test_serve_config_errors_without_gpu_work():
    L = _lib.lib()
    srv = C.c_void_p()
    cfg = _lib.ServeCfg()
    cfg.opts = L.drk_opts_default()
    cfg.max_inflight = 0
    cfg.queue_capacity = 16
    assert L.drk_serve_create(C.byref(cfg), C.byref(srv)) == _lib.DRK_EINVAL       # no slots
    cfg.max_inflight = 4
    cfg.queue_capacity = 0
    assert L.drk_serve_create(C.byref(cfg), C.byref(srv)) == _lib.DRK_EINVAL       # no queue
    cfg.queue_capacity = 16
    cfg.opts.cache_len = 9
    assert L.drk_serve_create(C.byref(cfg), C.byref(srv)) == _lib.DRK_EINVAL       # cache too long
    assert L.drk_serve_submit(None, 0, None, None, None) == _lib.DRK_EINVAL
    assert L.drk_serve_poll(None, 1, 0, None) == _lib.DRK_EINVAL


def test_ctypes_structs_match_the_header(tmp_path):
    """The binding's ctypes structs have the sizes and field offsets that a C compiler gives the
    header's structs (compiled here with the host C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = {"drk_scene": _lib.Scene, "drk_scene_grad": _lib.SceneGrad, "drk_scene_out": _lib.SceneOut,
             "drk_camera": _lib.Camera, "drk_opts": _lib.Opts, "drk_serve_cfg": _lib.ServeCfg,
             "drk_req_stats": _lib.ReqStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-o", str(exe), str(src)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, val = ln.split()
        got[(cname, field)] = int(val)
    for cname, py in pairs.items():
        assert C.sizeof(py) == got[(cname, "size")], cname
        for fname, _ in py._fields_:
            assert getattr(py, fname).offset == got[(cname, fname)], (cname, fname)
