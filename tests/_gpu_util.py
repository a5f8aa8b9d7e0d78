"""Shared helpers of the GPU parity tests (HIP path vs FP64 oracle)."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import drk_oracle as O

IMG_TOL = 1e-4            # per colour channel, FP32 path vs FP64 oracle (unflagged pixels)
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


def gpu_opts(cache_len=8, lowpass=True, cull_mode=0, key_mode=0):
    from paper_2412_11752_amd import make_opts
    return make_opts(lowpass_sl=math.sqrt(0.5) if lowpass else 0.0, cache_len=cache_len, cull_mode=cull_mode,
                     key_mode=key_mode)


def oracle_flat_lists(tiles):
    t_out, j_out = [], []
    for t in sorted(tiles):
        for _, j in tiles[t]:
            t_out.append(t)
            j_out.append(j)
    return np.array(t_out, np.int64), np.array(j_out, np.int64)


def compare_image(gpu_rgb_chw, orc, H, W, tol=IMG_TOL):
    """gpu (3, H, W) vs oracle PixelResult (H*W, 3).  Returns (max err unflagged, #flagged, max flagged)."""
    g = gpu_rgb_chw.reshape(3, H * W).T.astype(np.float64)
    err = np.abs(g - orc.rgb).max(axis=1)
    knife = orc.knife
    ok = err[~knife]
    return (float(ok.max()) if ok.size else 0.0), int(knife.sum()), (float(err[knife].max()) if knife.any() else 0.0), err
