"""Shared helpers of the GPU parity tests (HIP path vs FP64 oracle)."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import drk_oracle as O

IMG_TOL = 1e-4            # per colour channel, FP32 path vs FP64 oracle (unflagged pixels)
KNIFE_TOL = 1.0 / 255.0 + 1e-4   # flagged pixels: one contribution near alpha_min may flip
KNIFE_MAX_FRAC = 1e-3     # pixels with a decision within 1e-6 of a threshold


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_opts(cache_len=8, lowpass=True, cull_mode=0, key_mode=0):
    return O.Opts(lowpass_sl=math.sqrt(0.5) if lowpass else 0.0, cache_len=cache_len, cull_mode=cull_mode,
                  key_mode=key_mode).f32()


def gpu_opts(cache_len=8, lowpass=True, cull_mode=0, key_mode=0, counters=0):
    from paper_2412_11752_amd import make_opts
    return make_opts(lowpass_sl=math.sqrt(0.5) if lowpass else 0.0, cache_len=cache_len, cull_mode=cull_mode,
                     key_mode=key_mode, counters=counters)


def oracle_flat_lists(tiles):
    t_out, j_out = [], []
    for t in sorted(tiles):
        for _, j in tiles[t]:
            t_out.append(t)
            j_out.append(j)
    return np.array(t_out, np.int64), np.array(j_out, np.int64)


def compare_image(gpu_rgb_chw, orc, H, W, tol=IMG_TOL, max_knife_frac=0.01):
    """gpu (3, H, W) vs oracle PixelResult (H*W, 3).  Asserts the bound on knife-edge pixels (within
    KNIFE_TOL, at most max_knife_frac of the image or 2 pixels); the caller asserts the unflagged
    bound.  Returns (max err unflagged, #flagged, max flagged, per-pixel err)."""
    g = gpu_rgb_chw.reshape(3, H * W).T.astype(np.float64)
    err = np.abs(g - orc.rgb).max(axis=1)
    knife = orc.knife
    ok = err[~knife]
    worst_k = float(err[knife].max()) if knife.any() else 0.0
    log(f"  {H}x{W}: {int(knife.sum())} knife-edge pixels, max err on them {worst_k:.3e}")
    assert worst_k <= KNIFE_TOL, f"knife-edge pixel off by {worst_k:.3e} (bound {KNIFE_TOL:.3e})"
    assert knife.sum() <= max(2, max_knife_frac * H * W), f"{int(knife.sum())} knife-edge pixels of {H * W}"
    return (float(ok.max()) if ok.size else 0.0), int(knife.sum()), worst_k, err


def compare_pixels(gpu_rgb_chw, orc, px, py, label="", max_knife_frac=0.01):
    """Sampled pixels (px, py) of a gpu (3, H, W) image vs the oracle's PixelResult for them: every
    unflagged pixel within IMG_TOL, every flagged one within KNIFE_TOL, and at most max_knife_frac
    of them (or 2) flagged.  Returns (worst unflagged, #flagged, worst flagged)."""
    err = np.abs(gpu_rgb_chw[:, py, px].T.astype(np.float64) - orc.rgb).max(axis=1)
    knife = orc.knife
    worst = float(err[~knife].max()) if (~knife).any() else 0.0
    worst_k = float(err[knife].max()) if knife.any() else 0.0
    log(f"{label}: {len(px)} px, max err {worst:.3e}, {int(knife.sum())} knife-edge px (max {worst_k:.3e}), "
        f"mean emitted {orc.n_emit.mean():.1f}")
    assert worst <= IMG_TOL, (label, worst)
    assert worst_k <= KNIFE_TOL, (label, worst_k)
    assert knife.sum() <= max(2, max_knife_frac * len(px)), (label, int(knife.sum()))
    return worst, int(knife.sum()), worst_k
