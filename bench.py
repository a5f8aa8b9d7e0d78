#!/usr/bin/env python3
"""Throughput of the DRK rasterizer on one MI355X.

Workload (default): 1M DRKs (K = 8, SH degree 3) in 64 anisotropic clusters of a 20-unit box,
rendered at 1920x1080 along a 100-frame camera path inside the box.  Inputs are resident in HBM
before the timed region starts.

  fwd phase     : per step one view: preprocess -> bin/sort -> forward raster   -> value (Mpix/s);
                  consecutive steps alternate over --streams workspaces and streams (default 3),
                  so one view's preprocess and sort overlap the previous views' rasters
  fwd+bwd phase : per step one view: the forward above + backward raster + per-primitive backward

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s fwd and fwd+bwd it/s at 1M DRKs 1080p; served p50/p99 latency vs plain"

# Algorithmic work per unit (see the design notes): FP32 operations with an FMA counted as 2 and an
# elementary function (reciprocal, exp, atan2, cospi) counted as 1.


def ops_hit(K: int) -> int:
    # every (pixel, primitive) evaluation behind the wave's box test: homography hit, depth and
    # grazing tests, low-pass reach, radius cut, pseudo-angle, sector search (2K), cross/dot
    # products, L1 radius and the energy lower bound with its cut
    return 63 + 2 * K


OPS_KERNEL = 27                # past both cuts: atan2, sin/cos(pi t/2), L2 weight, energy, exp, Psi, low-pass, clamp
OPS_CACHE = 49                 # per contributor: 7 key compares + 2 selects per slot for key, alpha, index
OPS_COMPOSITE = 10             # per emitted contribution: transmittance test and colour update
VALU_PEAK_TFLOPS = 157.3                          # MI355X published FP32 vector peak (packed FMA counted as 2)
VALU_NONPACKED_TFLOPS = 256 * 64 * 2.4e9 * 2 / 1e12   # 78.6: one FMA per lane per clock (the build emits no packed FP32)
HBM_PEAK_GBS = 8000.0


def preprocess_bytes(n, visible, K, ncol):
    """Algorithmic HBM bytes of the preprocess per view: every primitive's geometry read once to cull
    it (centre, rotation, K scales and angles, eta, tau, opacity) and its key and tile count written;
    each visible primitive's parameters read again with its colour, and its render record written."""
    geo = 4 * (3 + 4 + 2 * K + 3)
    rec = 4 * ((36 + 8 * K + 3) & ~3)
    return n * (geo + 8) + visible * (geo + 4 * ncol + rec)


def bin_sort_bytes(visible, pairs, tiles):
    """Algorithmic HBM bytes of the bin/sort per view as implemented: compaction of the visible set
    (key + index written), four 8-bit passes of the stable depth sort and the pair sort's passes
    (each reads the keys twice and the values once and writes both: 20 B per element), the
    duplication (8 B per pair written), the ranges (4 B per pair read)."""
    tile_passes = (max(1, (tiles - 1).bit_length()) + 7) // 8
    return visible * 8 + visible * 20 * 4 + pairs * 8 + pairs * 20 * tile_passes + pairs * 4


def raster_traffic():
    """HBM bytes per raster launch measured with rocprofv3 counters (profiles/), or None when the
    raster sources have changed since that measurement."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", "render_fwd_c3_1080p_traffic.md")).read()
    except OSError:
        return None
    m_t = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    m_h = re.search(r"raster_sources_sha256: ([0-9a-f]+)", text)
    h = hashlib.sha256()
    for name in ("render_fwd.hip", "raster_common.hpp", "drk_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2412_11752_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if not (m_t and m_h) or m_h.group(1) != h.hexdigest():
        return None
    return int(m_t.group(1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sized_rasterizer(ds, frames, W, H, opts, count=1):
    """`count` rasterizers whose pair buffers fit every frame of the list (sized in an untimed pass)."""
    from paper_2412_11752_amd import Rasterizer
    ras = Rasterizer(ds.n, ds.K, W, H, pair_capacity=1 << 26)
    need = 0
    for cam in frames:
        ras.preprocess(ds, [cam], opts)
        ras.bin_sort()
        _, nd = ras.status()
        need = max(need, nd)
    cap = int(need * 1.05) + 4096
    ras.close()
    out = [Rasterizer(ds.n, ds.K, W, H, pair_capacity=cap) for _ in range(count)]
    return (out[0] if count == 1 else out), cap, need


class Lane:
    """One in-flight frame slot: a workspace, its output buffers and its stream."""

    def __init__(self, ras, W, H, stream):
        import torch
        self.ras, self.stream = ras, stream
        self.rgb = torch.empty(3 * W * H, device="cuda")
        self.T = torch.empty(W * H, device="cuda")


def make_lanes(ras_list, W, H):
    """Frame slots: the first on the current stream, the others on their own default-priority
    streams (consecutive frames are independent, so slot i % n renders frame i)."""
    import torch
    return [Lane(r, W, H, torch.cuda.current_stream() if i == 0 else torch.cuda.Stream())
            for i, r in enumerate(ras_list)]


def timed(lanes, ds, frames, opts, args, bwd=False):
    """Times args.steps frames (after args.warmup untimed ones), frame i on lane i % len(lanes);
    per-stage HIP events on each frame's stream.  Returns (wall seconds, [steps][4] ms: preprocess,
    bin/sort, fwd, bwd)."""
    import torch
    from paper_2412_11752_amd._lib import DRK_OK, DrkError
    g_up = [torch.full_like(ln.rgb, 0.01) for ln in lanes] if bwd else None

    def frame(i, e=None):
        k = i % len(lanes)
        ln = lanes[k]
        with torch.cuda.stream(ln.stream):
            if e: e[0].record(ln.stream)
            ln.ras.preprocess(ds, [frames[i]], opts)
            if e: e[1].record(ln.stream)
            ln.ras.bin_sort()
            if e: e[2].record(ln.stream)
            ln.ras.render_fwd(ln.rgb, ln.T)
            if e: e[3].record(ln.stream)
            if bwd:
                ln.ras.render_bwd(ln.rgb, g_up[k])
            if e: e[4].record(ln.stream)
    for i in range(args.warmup):
        frame(i)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        frame(args.warmup + s, ev[s])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3]),
                    e[3].elapsed_time(e[4])] for e in ev])
    for ln in lanes:
        with torch.cuda.stream(ln.stream):
            code, _ = ln.ras.status()
        if code != DRK_OK:
            raise DrkError(code, "timed loop")
    return t_total, ms


def raster_work(ras, ds, frames, opts, args, rgb, T):
    # (sequential, on the current stream: the counts do not depend on timing)
    """Work units of the forward raster per launch, averaged over the timed frames (re-rendered:
    the pipeline is deterministic), counted by the kernel itself."""
    tot = dict(listed=0, hits=0, kernels=0, contributors=0, emitted=0)
    pairs, visible = [], []
    names = dict(listed="consumed", hits="hits", kernels="kernels", contributors="contributors", emitted="emitted")
    counted = type(opts).from_buffer_copy(opts)
    counted.counters = 1          # the instrumented launch writes the per-pixel work counters
    for s in range(args.steps):
        ras.preprocess(ds, [frames[args.warmup + s]], counted)
        ras.bin_sort()
        ras.render_fwd(rgb, T)
        for k, e in names.items():
            tot[k] += int(ras.export(e).sum().item())
        pairs.append(ras.status()[1])
        visible.append(int((ras.export("tile_counts") != 0).sum().item()))
    out = {k: v // args.steps for k, v in tot.items()}
    out["pairs_max"], out["pairs_mean"] = int(max(pairs)), float(np.mean(pairs))
    out["visible_mean"] = float(np.mean(visible))
    out["flops"] = (tot["hits"] * ops_hit(ds.K) + tot["kernels"] * OPS_KERNEL + tot["contributors"] * OPS_CACHE
                    + tot["emitted"] * OPS_COMPOSITE) / args.steps
    return out


def c3_small_phase(args, ds, opts):
    """The 1M-DRK cluster scene at 1297x840 along the same camera path (the 1297x840 image size of the
    training-step workload): forward Mpix/s with the bench's frames in flight and with one."""
    from drk_synth import c3_camera_path
    W, H = 1297, 840
    cams = c3_camera_path(202, 100, W, H, half=10.0)
    frames = [cams[i % len(cams)] for i in range(args.warmup + args.steps)]
    rl, cap, need = sized_rasterizer(ds, frames, W, H, opts, count=args.streams)
    rl = rl if isinstance(rl, list) else [rl]
    lanes = make_lanes(rl, W, H)
    from paper_2412_11752_amd import make_opts
    t_total, ms = timed(lanes, ds, frames, make_opts(launch_order=1) if len(lanes) > 1 else opts, args)
    t1, ms1 = timed(lanes[:1], ds, frames, opts, args)
    out = {"width": W, "height": H, "mpix_s": round(args.steps * W * H / t_total / 1e6, 2),
           "ms_per_step": round(t_total * 1e3 / args.steps, 4), "frames_in_flight": len(lanes),
           "one_frame_mpix_s": round(args.steps * W * H / t1 / 1e6, 2),
           "ms_breakdown": {k: round(float(ms1[:, i].mean()), 4) for i, k in
                            enumerate(["preprocess", "bin_sort", "render_fwd"])}, "pairs_max": need}
    log(f"c3 1297x840: {out}")
    for r in rl:
        r.close()
    return out


def c5_phase(args, opts):
    """3M DRKs (K = 16, SH3) in 64 clusters of a 40-unit box, eight 1920x1080 views per step in one
    call with per-view sort buffers: Mpix/s of the forward and the device memory it holds."""
    import torch
    from drk_synth import config_c5
    from paper_2412_11752_amd import DRKScene, Rasterizer
    t0 = time.time()
    scene, cams = config_c5()
    ds = DRKScene.from_host(scene, device="cuda")
    log(f"c5: {scene.n} DRKs K={scene.K}, {scene.nbytes() / 1e9:.2f} GB, gen {time.time() - t0:.1f}s")
    W, H, V = cams[0].width, cams[0].height, len(cams)
    probe = Rasterizer(scene.n, scene.K, W, H, max_views=V, pair_capacity=1 << 24)
    probe.preprocess(ds, cams, opts)
    probe.bin_sort()
    need = probe.status()[1]
    probe.close()
    torch.cuda.empty_cache()
    cap = int(need * 1.05) + 4096
    free0, total = torch.cuda.mem_get_info()
    ras = Rasterizer(scene.n, scene.K, W, H, max_views=V, pair_capacity=cap)
    rgb = torch.empty(V * 3 * W * H, device="cuda")
    T = torch.empty(V * W * H, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(max(1, args.warmup)):
        ras.preprocess(ds, cams, opts)
        ras.bin_sort()
        ras.render_fwd(rgb, T)
    steps = max(2, args.steps // 4)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    t_s = time.perf_counter()
    stage = np.zeros(3)
    for _ in range(steps):
        ev[0].record(stream)
        ras.preprocess(ds, cams, opts)
        ev[1].record(stream)
        ras.bin_sort()
        ev[2].record(stream)
        ras.render_fwd(rgb, T)
        ev[3].record(stream)
        torch.cuda.synchronize()
        stage += [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])]
    dt = time.perf_counter() - t_s
    free1, _ = torch.cuda.mem_get_info()
    code, _ = ras.status()
    out = {"n_prims": scene.n, "K": scene.K, "views": V, "width": W, "height": H,
           "mpix_s": round(steps * V * W * H / dt / 1e6, 2), "ms_per_step": round(dt * 1e3 / steps, 3),
           "ms_breakdown": {k: round(float(v) / steps, 3) for k, v in zip(["preprocess", "bin_sort", "render_fwd"], stage)},
           "pairs_all_views_max": need, "scene_bytes": scene.nbytes(),
           "workspace_bytes": Rasterizer.size_query(scene.n, scene.K, W, H, V, cap),
           "device_bytes_in_use": int(total - free1), "device_bytes_before_workspace": int(total - free0),
           "status": int(code), "fwd_bwd_it_per_s": None}
    log(f"c5: {out}")
    ras.close()
    del ds, rgb, T
    torch.cuda.empty_cache()
    return out


def ksweep_phase(args, opts, W, H):
    """Rendering cost against the number of radial bases K (the cost side of the K ablation): the
    same cluster centres and orientations, scales and angles drawn for each K, same camera path."""
    import torch
    from drk_synth import c3_camera_path, scene_clusters
    from paper_2412_11752_amd import DRKScene
    out = {}
    cams = c3_camera_path(202, 100, W, H, half=10.0)
    frames = [cams[i % len(cams)] for i in range(args.warmup + args.steps)]
    for K in [int(k) for k in args.ksweep.split(",")]:
        t0 = time.time()
        host = scene_clusters(2, args.n, K=K, half=10.0)
        ds = DRKScene.from_host(host, device="cuda")
        # one frame in flight: the per-stage times compare K without overlap between frames
        ras, cap, need = sized_rasterizer(ds, frames, W, H, opts)
        rl = [ras]
        lanes = make_lanes(rl, W, H)
        t_total, ms = timed(lanes, ds, frames, opts, args)
        work = raster_work(ras, ds, frames, opts, args, lanes[0].rgb, lanes[0].T)
        raster_ms = float(ms[:, 2].mean())
        row = {"mpix_s": round(args.steps * W * H / t_total / 1e6, 2),
               "ms_preprocess": round(float(ms[:, 0].mean()), 4), "ms_bin_sort": round(float(ms[:, 1].mean()), 4),
               "ms_raster": round(raster_ms, 4), "pairs_max": need,
               "hits": work["hits"], "kernels": work["kernels"], "contributors": work["contributors"],
               "emitted": work["emitted"], "raster_tflops": round(work["flops"] / raster_ms / 1e9, 3),
               "ns_per_hit": round(raster_ms * 1e6 / max(work["hits"], 1), 4)}
        log(f"ksweep K={K}: {row} (scene gen + sizing {time.time() - t0:.1f}s)")
        out[str(K)] = row
        for r in rl:
            r.close()
        del ds
        torch.cuda.empty_cache()
    return out


def sortacc_phase(args, lanes, ds, frames, W, H):
    """Sorting accuracy of the pre-sort keys (supplement, cache-sorting evaluation): randomly placed
    and oriented kernels (1500 DRKs, K = 8, scales 0.05-0.5 in a 2-unit box) rendered at 512x512
    with each key and cache length, traced front to back and measured by drk_trace_metrics, and
    each image compared with the exact per-pixel order's; plus the cost of each key on the headline
    workload (same frames as the fwd phase)."""
    import torch
    from drk_synth import camera_lookat, scene_uniform_box
    from paper_2412_11752_amd import DRKScene, Rasterizer, make_opts, trace_metrics
    out = {"scene": "1500 DRKs (K=8) uniform in [-1,1]^3, scales log-uniform in [0.05, 0.5], random orientations, "
                    "512x512 view from distance 3", "cap": 64, "metrics": {}, "cost": {}}
    host = scene_uniform_box(77, 1500, K=8, half=1.0, s_lo=0.05, s_hi=0.5)
    cam = camera_lookat((0.4, -0.3, -3.0), (0, 0, 0), (0, 1, 0), 512, 512, 60.0, bg=(0.1, 0.1, 0.1))
    sd = DRKScene.from_host(host, device="cuda")
    r2 = Rasterizer(host.n, host.K, 512, 512, pair_capacity=1 << 22)
    names = {0: "centre", 1: "centric", 2: "nearest"}
    # the exact per-pixel order (cache_len >= 2^30) as the reference image
    exact_opts = make_opts(cache_len=1 << 30)
    r2.preprocess(sd, [cam], exact_opts)
    r2.bin_sort()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(torch.cuda.current_stream())
    ref, _ = r2.render_fwd()
    e1.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    out["exact_ms"] = round(e0.elapsed_time(e1), 3)
    out["image_vs_exact"] = {}
    for mode in (0, 1, 2):
        row, img = {}, {}
        for L in (1, 2, 4, 8):
            r2.preprocess(sd, [cam], make_opts(cache_len=L, key_mode=mode))
            r2.bin_sort()
            _, _, tn, ti, tz = r2.render_trace(64)
            m = trace_metrics(tn, tz, 64)
            row[str(L)] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in m.items()}
            rgb, _ = r2.render_fwd()
            d = (rgb - ref).abs()
            mse = float((d * d).mean())
            img[str(L)] = {"mean_abs": round(float(d.mean()), 6), "max_abs": round(float(d.max()), 5),
                           "psnr_db": round(10 * math.log10(1.0 / mse), 2) if mse > 0 else None}
        out["metrics"][names[mode]] = row
        out["image_vs_exact"][names[mode]] = img
        log(f"sortacc {names[mode]}: " + ", ".join(f"L={L} acc {v['accuracy']:.3f} tau {v['kendall_tau']:.3f} "
                                                  f"mae {v['mae']:.4f} psnr-vs-exact {img[L]['psnr_db']}"
                                                  for L, v in row.items()))
    r2.close()
    for mode in (0, 1, 2):
        t_total, ms = timed(lanes[:1], ds, frames, make_opts(key_mode=mode), args)   # one frame in flight
        out["cost"][names[mode]] = {"mpix_s": round(args.steps * W * H / t_total / 1e6, 2),
                                    "ms_preprocess": round(float(ms[:, 0].mean()), 4),
                                    "ms_bin_sort": round(float(ms[:, 1].mean()), 4),
                                    "ms_raster": round(float(ms[:, 2].mean()), 4)}
        log(f"sortacc cost {names[mode]}: {out['cost'][names[mode]]}")
    return out


def mesh_phase(args, W, H):
    """Mesh to DRK (section "Converting Mesh to DRK"): a 917k-face scene of 64 randomly placed
    icospheres (20480 triangles) and tori (8192 quads) converted on the GPU with K = 4, then rendered
    at W x H with the depth and normal channels, for each pre-sort key; plus the sorting accuracy of
    each key on it (traced, first 64 composited contributions per pixel)."""
    import torch
    from drk_synth import camera_lookat, mesh_scene
    from paper_2412_11752_amd import Rasterizer, make_opts, mesh_to_drk, trace_metrics
    V, F, C = mesh_scene(5, n_instances=64, ico_level=5, torus=(128, 64), half=3.0)
    v = torch.as_tensor(np.ascontiguousarray(V.T, np.float32), device="cuda")
    f = torch.as_tensor(np.ascontiguousarray(F, np.int32), device="cuda")
    c = torch.as_tensor(np.ascontiguousarray(C.T), device="cuda")
    ds, rej = mesh_to_drk(v, f, c, 4, 0.95, 0.99)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        ds, rej = mesh_to_drk(v, f, c, 4, 0.95, 0.99)
    e1.record(stream)
    torch.cuda.synchronize()
    out = {"scene": f"{F.shape[0]} faces (64 icospheres of 20480 triangles and tori of 8192 quads in a 6-unit box), K=4",
           "convert_ms": round(e0.elapsed_time(e1) / 10, 4), "rejected": rej, "render": {}, "sortacc": {}}
    log(f"mesh: {F.shape[0]} faces converted in {out['convert_ms']:.3f} ms ({rej} rejected)")
    cams = [camera_lookat((9.0 * math.cos(a), 1.5, 9.0 * math.sin(a)), (0, 0, 0), (0, 1, 0), W, H, 60.0)
            for a in np.linspace(0, 2 * math.pi, args.warmup + args.steps, endpoint=False)]
    ras = Rasterizer(ds.n, 4, W, H, pair_capacity=1 << 25)
    names = {0: "centre", 1: "centric", 2: "nearest"}
    for mode in (0, 1, 2):
        opts = make_opts(key_mode=mode)
        for i in range(args.warmup):
            ras.preprocess(ds, [cams[i]], opts)
            ras.bin_sort()
            ras.render_depth_normal()
        code, need = ras.status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            ras.preprocess(ds, [cams[args.warmup + i]], opts)
            ras.bin_sort()
            ras.render_depth_normal()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        code, need = ras.status()
        out["render"][names[mode]] = {"mpix_s": round(args.steps * W * H / dt / 1e6, 2), "pairs": need,
                                      "status": int(code)}
        row = {}
        for L in (1, 8):
            ras.preprocess(ds, [cams[args.warmup]], make_opts(key_mode=mode, cache_len=L))
            ras.bin_sort()
            _, _, tn, ti, tz = ras.render_trace(64)
            m = trace_metrics(tn, tz, 64)
            row[str(L)] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in m.items()}
            del tn, ti, tz
        out["sortacc"][names[mode]] = row
        log(f"mesh {names[mode]}: {out['render'][names[mode]]}, L=1 acc {row['1']['accuracy']:.3f} tau "
            f"{row['1']['kendall_tau']:.4f}, L=8 acc {row['8']['accuracy']:.3f} tau {row['8']['kendall_tau']:.4f}")
    ras.close()
    return out


def train_phase(args):
    """Parametrization and optimizer kernels at the headline size (1M DRKs, K = 8, SH3: 74 floats
    each), raw parameters laid out in one flat buffer so one Adam launch updates all of them.
    Algorithmic bytes per DRK: activation reads 74 and writes 74 floats; its VJP reads the 23 raw
    floats it needs (q, s, theta, eta, tau, o) and 74 gradients and writes 74; Adam reads p, m, v,
    g and writes p, m, v (28 B per float).  The raster backward these would feed is switched off."""
    import torch
    from paper_2412_11752_amd import DRKScene, activate, activate_bwd, adam_step
    n, K, ncol = args.n, 8, 48
    rows = [("mu", 3), ("q", 4), ("scale", K), ("theta", K), ("eta", 1), ("tau", 1), ("opacity", 1), ("color", ncol)]
    total = sum(r for _, r in rows) * n
    g = torch.Generator(device="cuda").manual_seed(9)
    flat = torch.randn(total, device="cuda", generator=g)
    gflat = torch.randn(total, device="cuda", generator=g) * 1e-3

    def views(buf):
        out, off = {}, 0
        for name, r in rows:
            t = buf[off:off + r * n]
            out[name] = t.view(r, n) if name not in ("eta", "tau", "opacity") else t
            off += r * n
        return DRKScene(out["mu"], out["q"], out["scale"], out["theta"], out["eta"], out["tau"], out["opacity"],
                        out["color"], 3)
    raw, gact = views(flat), views(gflat)
    m = torch.zeros_like(flat)
    v = torch.zeros_like(flat)
    stream = torch.cuda.current_stream()
    res = {}

    def time_it(name, fn, nbytes, reps=20):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = nbytes / (ms / 1e3) / 1e9
        res[name] = {"ms": round(ms, 4), "bytes": int(nbytes), "GB_s": round(gbs, 1), "frac_hbm": round(gbs / 8000.0, 3)}
        log(f"train {name}: {ms:.4f} ms, {gbs:.0f} GB/s ({gbs / 8000.0:.2f} of 8 TB/s)")
    fl = 74
    time_it("activate", lambda: activate(raw), n * fl * 8)
    time_it("activate_bwd", lambda: activate_bwd(raw, gact), n * (23 + fl + fl) * 4)
    step = [0]

    def adam():
        step[0] += 1
        adam_step(flat, m, v, gflat, 5e-3, 0.9, 0.999, 1e-15, step[0])
    time_it("adam", adam, total * 28)
    return {"n_prims": n, "floats_per_prim": fl, "kernels": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--phases", default="fwd,c3small,c5,serve",
                    help="fwd, fwdbwd (backward switched off), c3small (1297x840), c5 (3M DRKs K=16, 8 views), "
                         "serve, ksweep, sortacc, mesh, train")
    ap.add_argument("--ksweep", default="3,5,8,16", help="radial basis counts of the ksweep phase")
    ap.add_argument("--streams", type=int, default=3,
                    help="frames in flight: consecutive frames alternate over this many workspaces and streams")
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="length of the headline Poisson trace")
    ap.add_argument("--serve-rates", default="200,800,1600,3200,6400",
                    help="request arrival rates (1/s): the first is the headline point, the rest the load sweep")
    ap.add_argument("--sweep-seconds", type=float, default=3.0, help="length of each sweep trace")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU oracle sample budget (0 = skip)")
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3 (no CPU baseline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the multi-GPU sharding is described in the design notes, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from drk_synth import config_c3
    from paper_2412_11752_amd import DRKScene, make_opts
    from paper_2412_11752_amd._lib import DrkError

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    W, H = args.width, args.height
    t0 = time.time()
    scene, cams = config_c3(n=args.n, width=W, height=H)
    log(f"scene: {scene.n} DRKs K={scene.K} SH{scene.sh_degree}, {scene.nbytes() / 1e6:.1f} MB; gen {time.time() - t0:.1f}s")
    ds = DRKScene.from_host(scene, device=dev)
    opts = make_opts()
    K = scene.K
    n_frames = args.warmup + args.steps
    frames = [cams[i % len(cams)] for i in range(n_frames)]

    rl, cap, need = sized_rasterizer(ds, frames, W, H, opts, count=args.streams)
    rl = rl if isinstance(rl, list) else [rl]
    lanes = make_lanes(rl, W, H)
    ras, rgb, T = rl[0], lanes[0].rgb, lanes[0].T
    log(f"pairs per view (max over frames): {need}  capacity {cap}; {len(lanes)} frame(s) in flight")
    result = {}

    phases = [p for p in args.phases.split(",") if p]
    # with frames in flight, row-major tile launch order leaves each raster's tail to the next frame's
    # preprocess; with one frame in flight the default (longest tile lists first) is faster
    opts_fwd = make_opts(launch_order=1) if len(lanes) > 1 else opts
    if "fwd" in phases:
        t_total, ms = timed(lanes, ds, frames, opts_fwd, args, bwd=False)
        mpix = args.steps * W * H / t_total / 1e6
        log(f"fwd: {t_total * 1e3 / args.steps:.3f} ms/step, {mpix:.1f} Mpix/s; "
            f"preprocess {ms[:, 0].mean():.3f} ms, bin/sort {ms[:, 1].mean():.3f} ms, raster {ms[:, 2].mean():.3f} ms")
        result["fwd"] = dict(t_total=t_total, ms=ms, mpix=mpix)
        if len(lanes) > 1 and not args.profile:
            t1, ms1 = timed(lanes[:1], ds, frames, opts, args, bwd=False)
            result["fwd1"] = dict(mpix=args.steps * W * H / t1 / 1e6, ms=ms1)
            log(f"fwd, one frame in flight: {t1 * 1e3 / args.steps:.3f} ms/step, {result['fwd1']['mpix']:.1f} Mpix/s; "
                f"raster {ms1[:, 2].mean():.3f} ms")
    if "fwdbwd" in phases:
        try:
            t_total, ms = timed(lanes, ds, frames, opts_fwd, args, bwd=True)
            its = args.steps / t_total
            log(f"fwd+bwd: {t_total * 1e3 / args.steps:.3f} ms/step, {its:.2f} it/s; bwd {ms[:, 3].mean():.3f} ms")
            result["fwdbwd"] = dict(t_total=t_total, ms=ms, its=its)
        except DrkError as e:
            log(f"fwd+bwd unavailable: {e}")

    work = raster_work(ras, ds, frames, opts, args, rgb, T)
    fwd = result.get("fwd")
    roofline, kernels_hbm = None, None
    if fwd is not None:
        # the raster's own launch time: from the one-frame-in-flight run (no other frame's kernels on
        # the GPU), HIP events on the stream the kernel is launched on
        one = result.get("fwd1", fwd)
        iso_ms = float(one["ms"][:, 2].mean())
        achieved = work["flops"] / (iso_ms / 1e3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / VALU_PEAK_TFLOPS, 4), "traffic": raster_traffic(),
                    "kernel": "k_render_fwd", "avg_launch_ms": round(iso_ms, 4),
                    "launch": "one frame in flight, longest tile lists first",
                    "peak_nonpacked": round(VALU_NONPACKED_TFLOPS, 1),
                    "frac_nonpacked": round(achieved / VALU_NONPACKED_TFLOPS, 4),
                    "flops_per_launch": int(work["flops"]),
                    "listed_pairs_per_launch": work["listed"],
                    "hit_evaluations_per_launch": work["hits"],
                    "kernel_evaluations_per_launch": work["kernels"],
                    "contributors_per_launch": work["contributors"],
                    "emitted_per_launch": work["emitted"]}
        if "fwd1" in result:
            fl_ms = float(fwd["ms"][:, 2].mean())
            # the same launches beside the other frames in flight (they share the CUs)
            roofline["in_flight"] = {"avg_launch_ms": round(fl_ms, 4),
                                     "achieved": round(work["flops"] / (fl_ms / 1e3) / 1e12, 3)}
        ncol = 3 * (scene.sh_degree + 1) ** 2 if scene.sh_degree >= 0 else 3
        tiles = ((W + 15) // 16) * ((H + 15) // 16)
        kernels_hbm = {}
        for name, col, nbytes in (
                ("preprocess", 0, preprocess_bytes(scene.n, work["visible_mean"], K, ncol)),
                ("bin_sort", 1, bin_sort_bytes(work["visible_mean"], work["pairs_mean"], tiles))):
            t = float(one["ms"][:, col].mean())
            gbs = nbytes / (t / 1e3) / 1e9
            kernels_hbm[name] = {"ms": round(t, 4), "bytes": int(nbytes), "GB_s": round(gbs, 1),
                                 "frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"raster work: {work['listed'] / 1e6:.1f}M listed, {work['hits'] / 1e6:.1f}M hits, "
            f"{work['kernels'] / 1e6:.1f}M kernel evaluations, {work['contributors'] / 1e6:.1f}M "
            f"contributors, {work['emitted'] / 1e6:.1f}M emitted per view -> {achieved:.2f} TFLOP/s "
            f"in {iso_ms:.3f} ms; preprocess / bin-sort HBM {kernels_hbm}")

    # CPU oracle on a bounded sample of the same workload (first timed frame)
    cpu = None
    if args.cpu_seconds > 0 and not args.profile:
        import torch as _t
        from oracle import drk_oracle as O
        ncores = os.cpu_count() or 1
        _t.set_num_threads(ncores)
        cam = frames[args.warmup]
        ras.preprocess(ds, [cam], opts)
        ras.bin_sort()
        ras.render_fwd(rgb, T)
        g = rgb.view(3, H, W).cpu().numpy()
        rng = np.random.default_rng(7)
        order = rng.permutation(W * H)
        done = 0
        errs = []
        t_c = time.perf_counter()
        oopts = O.Opts().f32()
        while time.perf_counter() - t_c < args.cpu_seconds and done < 4096:
            idx = order[done:done + 32]
            px, py = idx % W, idx // W
            r = O.render_pixels(scene, cam, oopts, px, py)
            e = np.abs(g[:, py, px].T - r.rgb).max(axis=1)
            errs.extend(e[~r.knife].tolist())
            done += idx.size
        el = time.perf_counter() - t_c
        cpu = {"value": round(done / el / 1e6, 9), "unit": "Mpix/s", "cores": _t.get_num_threads(),
               "kind": "oracle", "sample": f"{done} seeded pixels of the first timed 1920x1080 view (every primitive "
                                          f"tested per pixel through a lossless bounding prefilter), {el:.1f} s",
               "parity_max_err": float(max(errs)) if errs else None}
        log(f"cpu oracle: {done} px in {el:.1f}s -> {cpu['value']:.2e} Mpix/s; max |gpu-oracle| {cpu['parity_max_err']}")

    sortacc = None
    if "sortacc" in phases:
        sortacc = sortacc_phase(args, lanes, ds, frames, W, H)
    for r in rl:
        r.close()
    del lanes
    torch.cuda.empty_cache()
    ksweep = None
    if "ksweep" in phases:
        ksweep = ksweep_phase(args, opts, W, H)
    train = None
    if "train" in phases:
        train = train_phase(args)
        torch.cuda.empty_cache()
    mesh = None
    if "mesh" in phases:
        mesh = mesh_phase(args, W, H)
        torch.cuda.empty_cache()
    c3_small = None
    if "c3small" in phases:
        c3_small = c3_small_phase(args, ds, opts)
    c5 = None
    if "c5" in phases:
        del ds
        torch.cuda.empty_cache()
        c5 = c5_phase(args, opts)
    serve = None
    if "serve" in phases and not args.profile:
        serve = serve_phase(args, opts)

    ms_step = fwd["t_total"] * 1e3 / args.steps if fwd else None
    line = {
        "metric": METRIC,
        "value": round(fwd["mpix"], 3) if fwd else None,
        "unit": "Mpix/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4) if ms_step else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{scene.n} DRKs (K={K}, SH3) in 64 anisotropic clusters of a 20-unit box, "
                               f"{W}x{H}, camera path inside the box, one view per step, {args.streams} consecutive "
                               f"frames in flight on separate streams",
                   "n_prims": scene.n, "K": K, "width": W, "height": H,
                   "pairs_per_view": {"max": work["pairs_max"], "mean": round(work["pairs_mean"], 1)},
                   "visible_per_view_mean": round(work["visible_mean"], 1),
                   "frames_in_flight": args.streams,
                   "launch_order": "row-major" if args.streams > 1 else "longest lists first",
                   "one_frame_launch_order": "longest lists first"},
        "one_frame_in_flight_mpix_s": round(result["fwd1"]["mpix"], 3) if "fwd1" in result else None,
        "fwd_bwd_it_per_s": round(result["fwdbwd"]["its"], 3) if "fwdbwd" in result else None,
        "fwd_bwd_note": None if "fwdbwd" in result else
        "not measured: drk_render_bwd is switched off (returns DRK_EDEVICE) until the cause of its "
        "illegal memory access on gfx950 is shown",
        "ms_breakdown": {k: round(float(result.get("fwd1", fwd)["ms"][:, i].mean()), 4) for i, k in
                         enumerate(["preprocess", "bin_sort", "render_fwd"])} if fwd else None,
        "roofline": roofline,
        "kernels_hbm": kernels_hbm,
        "cpu_baseline": cpu,
        "serve": serve,
    }
    if c3_small is not None:
        line["c3_1297x840"] = c3_small
    if c5 is not None:
        line["c5_3m_k16_8x1080p"] = c5
    if ksweep is not None:
        line["ksweep"] = ksweep
    if sortacc is not None:
        line["sortacc"] = sortacc
    if mesh is not None:
        line["mesh"] = mesh
    if train is not None:
        line["train"] = train
    if "fwdbwd" in result:
        line["ms_breakdown"]["render_bwd"] = round(float(result["fwdbwd"]["ms"][:, 3].mean()), 4)
    print(json.dumps(line), flush=True)


def serve_phase(args, opts):
    """Continuous-batching server vs the plain sequential renderer on the same Poisson traces: 16
    resident scenes of 50k-1M DRKs, resolutions drawn from {256^2, 800^2, 1297x840, 1920x1080}.  The
    first rate is the headline point (its trace --serve-seconds long); the others sweep the offered
    load past the plain renderer's saturation (--sweep-seconds each)."""
    import torch
    from drk_synth import camera_from_yaw_pitch, config_c4_scenes
    from paper_2412_11752_amd import DRKScene, Rasterizer
    from paper_2412_11752_amd._lib import DRK_EAGAIN, check
    from paper_2412_11752_amd.serving import Server

    torch.cuda.empty_cache()   # the earlier phases' cached blocks
    t0 = time.time()
    hosts = config_c4_scenes()
    scenes = [DRKScene.from_host(h, device="cuda") for h in hosts]
    log(f"serve: {len(scenes)} scenes, {sum(h.n for h in hosts) / 1e6:.2f}M DRKs total, gen {time.time() - t0:.1f}s")
    res = [(256, 256), (800, 800), (1297, 840), (1920, 1080)]
    rng = np.random.default_rng(33)

    def trace(rate, seconds):
        n_req = max(1, int(seconds * rate))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
        which = rng.integers(0, len(scenes), n_req)
        rsel = rng.integers(0, len(res), n_req)
        cams = []
        for i in range(n_req):
            W, H = res[rsel[i]]
            pos = rng.uniform(-8.0, 8.0, 3)
            cams.append(camera_from_yaw_pitch(pos, rng.uniform(0, 2 * math.pi), math.radians(rng.uniform(-30, 30)),
                                              W, H))
        return arrivals, which, cams

    srv = Server(max_inflight=8, use_graphs=True, opts=opts, queue_capacity=1 << 16)
    sids = [srv.add_scene(d) for d in scenes]
    # warm every (scene, resolution) workspace and graph once, untimed
    for si in range(len(scenes)):
        for (W, H) in res:
            cam = camera_from_yaw_pitch((0.0, 0.0, 0.0), 0.3, 0.1, W, H)
            out = torch.empty(3 * W * H, device="cuda")
            srv.wait(srv.submit(sids[si], cam, out))
    rasters = {}

    def plain(which_i, cam):
        key = (which_i, cam.width, cam.height)
        if key not in rasters:
            h = hosts[which_i]
            rasters[key] = Rasterizer(h.n, h.K, cam.width, cam.height, pair_capacity=1 << 22)
        rgb, _ = rasters[key].forward(scenes[which_i], [cam], opts)
        return rgb

    for si in range(len(scenes)):         # warm the plain renderer's workspaces too
        for (W, H) in res:
            plain(si, camera_from_yaw_pitch((0.0, 0.0, 0.0), 0.3, 0.1, W, H))
    torch.cuda.synchronize()

    ring_len = 512     # output buffers per resolution, reused once their request is done

    def run_served(arrivals, which, cams, keep=()):
        """Replays the trace; returns copies of the outputs of the requests in `keep`.  Outputs come
        from a ring per resolution: a slot is reused once its previous request is done (a client
        that runs out of buffers waits, as it does on a full queue), so device memory stays bounded
        however long the trace."""
        n_req = len(cams)
        rids, stats, kept = [0] * n_req, [None] * n_req, {}
        rings = {r: [torch.empty(3 * r[0] * r[1], device="cuda") for _ in range(ring_len)] for r in res}
        owner = {r: [-1] * ring_len for r in res}
        count = {r: 0 for r in res}

        def finish(i, buf):
            stats[i] = srv.wait(rids[i])
            if i in keep:
                kept[i] = buf.clone()

        t_base = time.perf_counter()
        for i in range(n_req):
            while time.perf_counter() - t_base < arrivals[i]:
                pass
            r = (cams[i].width, cams[i].height)
            slot = count[r] % ring_len
            count[r] += 1
            buf = rings[r][slot]
            if owner[r][slot] >= 0:
                finish(owner[r][slot], buf)
            owner[r][slot] = i
            while True:                      # a full queue pushes back on the client
                code, rids[i] = srv.try_submit(sids[which[i]], cams[i], buf)
                if code != DRK_EAGAIN:
                    break
                time.sleep(50e-6)
            check(code, "drk_serve_submit")
        for r in res:
            for slot, i in enumerate(owner[r]):
                if i >= 0 and stats[i] is None:
                    finish(i, rings[r][slot])
        lat = np.array([(st["done_us"] - st["submit_us"]) / 1e3 for st in stats])
        span = (max(st["done_us"] for st in stats) - min(st["submit_us"] for st in stats)) / 1e6
        mpix = sum(st["width"] * st["height"] for st in stats) / 1e6
        del rings
        return kept, {"mpix_s": round(mpix / span, 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3), "makespan_s": round(span, 3),
                      "failed": int(sum(st["status"] != 0 for st in stats))}, mpix

    def run_plain(arrivals, which, cams, mpix):
        n_req = len(cams)
        done = np.zeros(n_req)
        t_base = time.perf_counter()
        for i in range(n_req):
            while time.perf_counter() - t_base < arrivals[i]:
                pass
            plain(which[i], cams[i])
            torch.cuda.synchronize()
            done[i] = time.perf_counter() - t_base
        lat = (done - arrivals) * 1e3
        span = done[-1] - arrivals[0]
        return {"mpix_s": round(float(mpix / span), 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "makespan_s": round(float(span), 3)}

    rates = [float(r) for r in args.serve_rates.split(",") if r]
    points, checked = [], 0
    for k, rate in enumerate(rates):
        seconds = args.serve_seconds if k == 0 else args.sweep_seconds
        arrivals, which, cams = trace(rate, seconds)
        pick = [int(i) for i in rng.choice(len(cams), min(12, len(cams)), replace=False)] if k == 0 else []
        outs, served, mpix = run_served(arrivals, which, cams, keep=set(pick))
        for i in pick:   # spot check: served results are bitwise the plain renderer's
            assert torch.equal(plain(which[i], cams[i]).reshape(-1), outs[i]), f"served request {i} differs"
            checked += 1
        del outs
        torch.cuda.synchronize()
        plain_res = run_plain(arrivals, which, cams, mpix)
        offered = mpix / float(arrivals[-1])
        pt = {"rate_per_s": rate, "trace_s": seconds, "requests": len(cams), "offered_mpix_s": round(offered, 2),
              "served": served, "plain_sequential": plain_res}
        # keeping up: the last result arrives within 10% (and 50 ms) of the end of the trace
        lim = 1.1 * float(arrivals[-1] - arrivals[0]) + 0.05
        pt["served_keeps_up"] = bool(served["makespan_s"] <= lim and served["failed"] == 0)
        pt["plain_keeps_up"] = bool(plain_res["makespan_s"] <= lim)
        log(f"serve {rate:.0f} req/s x {seconds:.0f}s ({len(cams)} requests, offered {offered:.0f} Mpix/s): "
            f"served {served}, plain {plain_res}")
        points.append(pt)
    srv.close()
    for r in rasters.values():
        r.close()
    head = points[0]
    keep = lambda key: max([p["rate_per_s"] for p in points if p[key]], default=None)
    return {"requests": head["requests"], "rate_per_s": head["rate_per_s"], "trace_s": head["trace_s"],
            "scenes": len(scenes), "resolutions": res, "served": head["served"],
            "plain_sequential": head["plain_sequential"], "bitwise_checked": checked,
            "sweep": points[1:], "max_rate_kept_up": {"served": keep("served_keeps_up"),
                                                      "plain_sequential": keep("plain_keeps_up")}}


if __name__ == "__main__":
    main()
