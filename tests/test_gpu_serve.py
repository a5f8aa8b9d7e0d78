"""Serving loop: continuous batching over resident scenes and mixed resolutions.

Each served result must be bitwise identical to the same request rendered alone (the forward pass is
deterministic), within 1e-4 of the oracle on a small request, and the admission errors must be
reported (queue full, never fits the budget, unknown scene)."""
import numpy as np
import pytest
import torch

from drk_synth import camera_lookat, config_c2, scene_uniform_box
from oracle import drk_oracle as O
from tests._gpu_util import IMG_TOL, compare_image, gpu_opts, log, need_gpu, oracle_opts

pytestmark = pytest.mark.gpu


def _cams(seed, sizes, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        az, el = rng.uniform(0, 2 * np.pi), rng.uniform(-0.5, 0.5)
        eye = 3.5 * np.array([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])
        W, H = sizes[i % len(sizes)]
        out.append(camera_lookat(eye, (0, 0, 0), (0, 0, 1), W, H, 60.0, bg=(0.05, 0.1, 0.15)))
    return out


@pytest.fixture(scope="module")
def scenes():
    need_gpu()
    from paper_2412_11752_amd import DRKScene
    hs = [config_c2(n=20_000)[0], scene_uniform_box(7, 5000, K=8), config_c2(n=60_000)[0]]
    return hs, [DRKScene.from_host(s) for s in hs]


@pytest.mark.parametrize("use_graphs", [True, False])
def test_mixed_requests_match_alone(scenes, use_graphs):
    from paper_2412_11752_amd import Rasterizer
    from paper_2412_11752_amd.serving import Server
    hs, ds = scenes
    sizes = [(64, 64), (200, 120), (331, 257), (800, 800)]
    cams = _cams(1, sizes, 24)
    srv = Server(max_inflight=4, use_graphs=use_graphs, opts=gpu_opts())
    ids = [srv.add_scene(d) for d in ds]
    outs, rids, which = [], [], []
    for i, cam in enumerate(cams):
        s = i % len(ids)
        out = torch.empty(3 * cam.height * cam.width, device="cuda")
        outs.append(out)
        which.append(s)
        rids.append(srv.submit(ids[s], cam, out))
    stats = [srv.wait(r) for r in rids]
    assert all(st["status"] == 0 for st in stats)
    overlap = sum(1 for a, b in zip(stats, stats[1:]) if b["start_us"] < a["done_us"])
    log(f"graphs={use_graphs}: {len(stats)} requests, {overlap} started before the previous finished")
    assert overlap >= 1        # the results below were produced in the mix, not one at a time
    torch.cuda.synchronize()
    for i, cam in enumerate(cams):
        h = hs[which[i]]
        ras = Rasterizer(h.n, h.K, cam.width, cam.height, pair_capacity=1 << 22)
        alone, _ = ras.forward(ds[which[i]], [cam], gpu_opts())
        assert torch.equal(alone.reshape(-1), outs[i]), i
    srv.close()


def test_served_request_matches_oracle(scenes):
    from paper_2412_11752_amd.serving import Server
    hs, ds = scenes
    cam = _cams(2, [(48, 40)], 1)[0]
    srv = Server(max_inflight=2, opts=gpu_opts())
    sid = srv.add_scene(ds[1])
    out = torch.empty(3 * 48 * 40, device="cuda")
    st = srv.wait(srv.submit(sid, cam, out))
    assert st["status"] == 0 and st["pairs"] > 0
    orc = O.render_image(hs[1], cam, oracle_opts())
    worst, nk, _, _ = compare_image(out.view(3, 40, 48).cpu().numpy(), orc, 40, 48)
    assert worst <= IMG_TOL
    srv.close()


def test_admission_errors(scenes):
    from paper_2412_11752_amd._lib import DRK_EAGAIN, DRK_ENOMEM, DRK_ENOTFOUND
    from paper_2412_11752_amd.serving import Server
    hs, ds = scenes
    cam = _cams(3, [(800, 800)], 1)[0]
    small = Server(hbm_budget_bytes=1 << 20, max_inflight=1, opts=gpu_opts())
    sid = small.add_scene(ds[0])
    out = torch.empty(3 * 800 * 800, device="cuda")
    code, _ = small.try_submit(sid, cam, out)
    assert code == DRK_ENOMEM
    code, _ = small.try_submit(sid + 5, cam, out)
    assert code == DRK_ENOTFOUND
    small.close()
    q = Server(max_inflight=1, queue_capacity=2, opts=gpu_opts())
    sid = q.add_scene(ds[2])
    codes = []
    rids = []
    bufs = [torch.empty(3 * 800 * 800, device="cuda") for _ in range(12)]
    for b in bufs:
        c, r = q.try_submit(sid, cam, b)
        codes.append(c)
        if c == 0:
            rids.append(r)
    assert DRK_EAGAIN in codes
    for r in rids:
        assert q.wait(r)["status"] == 0
    q.close()


def test_overflow_is_retried_with_a_larger_workspace(scenes):
    """A workspace whose first capacity guess is too small is regrown and the request re-run."""
    from paper_2412_11752_amd import Rasterizer
    from paper_2412_11752_amd.serving import Server
    hs, ds = scenes
    cam = _cams(4, [(800, 800)], 1)[0]
    cam_near = camera_lookat((0, 0, -1.6), (0, 0, 0), (0, 1, 0), 800, 800, 90.0)
    srv = Server(max_inflight=1, opts=gpu_opts(), initial_pairs=1000)
    sid = srv.add_scene(ds[2])
    out = torch.empty(3 * 800 * 800, device="cuda")
    st = srv.wait(srv.submit(sid, cam_near, out))
    assert st["status"] == 0 and st["pairs"] > 1000
    ras = Rasterizer(hs[2].n, hs[2].K, 800, 800, pair_capacity=1 << 20)
    alone, _ = ras.forward(ds[2], [cam_near], gpu_opts())
    assert torch.equal(alone.reshape(-1), out)
    srv.close()


def test_overflow_past_the_budget_is_reported(scenes):
    """A request whose first workspace fits the budget but whose pairs overflow it needs a larger
    workspace than the whole budget: the request completes with DRK_ENOMEM instead of waiting
    forever, and requests behind it still run."""
    from paper_2412_11752_amd import Rasterizer
    from paper_2412_11752_amd._lib import DRK_ENOMEM
    from paper_2412_11752_amd.serving import Server
    hs, ds = scenes
    cam_near = camera_lookat((0, 0, -1.6), (0, 0, 0), (0, 1, 0), 800, 800, 90.0)
    small = Rasterizer.size_query(hs[2].n, hs[2].K, 800, 800, 1, 1000)
    big = Rasterizer.size_query(hs[2].n, hs[2].K, 800, 800, 1, 200_000)
    assert big > small
    srv = Server(hbm_budget_bytes=(small + big) // 2, max_inflight=1, opts=gpu_opts(), initial_pairs=1000)
    sid = srv.add_scene(ds[2])
    out = torch.empty(3 * 800 * 800, device="cuda")
    st = srv.wait(srv.submit(sid, cam_near, out))
    log(f"overflowing request past the budget: status {st['status']}, pairs needed {st['pairs']}")
    assert st["status"] == DRK_ENOMEM and st["pairs"] > 200_000
    sid1 = srv.add_scene(ds[1])
    cam = _cams(5, [(64, 64)], 1)[0]
    out1 = torch.empty(3 * 64 * 64, device="cuda")
    assert srv.wait(srv.submit(sid1, cam, out1))["status"] == 0
    srv.close()


def test_small_requests_pass_a_waiting_large_one(scenes):
    """The budget holds one 800x800 workspace and a few small ones.  A second 800x800 request of the
    same scene needs a second such workspace and waits for the first request to finish; small
    requests submitted after it are admitted meanwhile (the waiting one is passed a bounded number
    of times), and every result equals the request rendered alone."""
    from paper_2412_11752_amd import Rasterizer
    from paper_2412_11752_amd.serving import Server
    hs, ds = scenes
    big_cam = camera_lookat((0, 0, -3.0), (0, 0, 0), (0, 1, 0), 800, 800, 60.0)
    small_cam = _cams(6, [(64, 64)], 1)[0]
    probe = Rasterizer(hs[2].n, hs[2].K, 800, 800, pair_capacity=1 << 24)
    probe.forward(ds[2], [big_cam], gpu_opts())
    need = probe.status()[1]
    probe.close()
    # a request that overflows is rerun with 25% (+1024) more pairs than it needed
    ws_big = Rasterizer.size_query(hs[2].n, hs[2].K, 800, 800, 1, need + need // 4 + 1024)
    ws_small = Rasterizer.size_query(hs[1].n, hs[1].K, 64, 64, 1, 1 << 17)
    budget = ws_big + 3 * ws_small + (1 << 20)
    assert 2 * ws_big > budget, (ws_big, ws_small)     # a second 800x800 workspace cannot fit beside the first
    srv = Server(hbm_budget_bytes=budget, max_inflight=4, opts=gpu_opts(), initial_pairs=0)
    sid = [srv.add_scene(d) for d in ds]
    warm = torch.empty(3 * 800 * 800, device="cuda")
    assert srv.wait(srv.submit(sid[2], big_cam, warm))["status"] == 0   # learns the 800x800 capacity
    jobs = [(2, big_cam), (2, big_cam)] + [(1, small_cam)] * 3
    outs, rids = [], []
    for s_i, cam in jobs:
        out = torch.empty(3 * cam.width * cam.height, device="cuda")
        outs.append(out)
        rids.append(srv.submit(sid[s_i], cam, out))
    stats = [srv.wait(r) for r in rids]
    assert all(st["status"] == 0 for st in stats)
    passed = sum(1 for st in stats[2:] if st["start_us"] < stats[1]["start_us"])
    log(f"budget {budget / 2**20:.1f} MiB (800x800 workspace {ws_big / 2**20:.1f}, 64x64 {ws_small / 2**20:.1f}): "
        f"{passed} of 3 small requests admitted before the waiting 800x800 one")
    assert stats[1]["start_us"] >= stats[0]["done_us"] - 1.0   # the second large request waited
    assert passed >= 1
    srv.close()
    for (s_i, cam), out in zip(jobs, outs):
        ras = Rasterizer(hs[s_i].n, hs[s_i].K, cam.width, cam.height, pair_capacity=need + 4096)
        alone, _ = ras.forward(ds[s_i], [cam], gpu_opts())
        assert torch.equal(alone.reshape(-1), out)
