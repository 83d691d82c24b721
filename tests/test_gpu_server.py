"""GPU tests of the served form (mls_server_*): requests of uneven size and
kind run concurrently on several slots, 16-bit Gaussian requests of one
kernel class batched into persistent kernels; every result is bit-identical
to the same fit run alone through mls_fit, and to the same request served
on a one-slot server.  Cancellation and timeouts, in the queue and inside a
running batch."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_requests(seed=0, count=12):
    from paper_1408_0677_amd import workloads as wl
    rng = np.random.default_rng(seed)
    reqs = []
    for q in range(count):
        n = int(rng.integers(200, 4000))
        d = int(rng.integers(1, 20))
        side = int(rng.integers(17, 200))
        basis = ["constant", "linear", "quadratic"][q % 3]
        prec = ["f64", "bf16", "fp16"][(q // 3) % 3]
        weight = "wendland" if (q % 4 == 3 and prec != "f64") else "gaussian"
        pts = wl.mixture_points(rng, n, k=3) if q % 2 else rng.random((n, 2))
        vals = rng.standard_normal((n, d))
        h = float(np.sqrt(30.0 / (np.pi * n))) * (2.0 if weight == "wendland" else 1.0)
        if prec != "f64":
            # 16-bit paths take tiles of at most 2.5 h (quadratic) / 4 h
            side = max(side, int(np.ceil(15.0 / (2.4 * h))))
        reqs.append(dict(pts=pts.astype(np.float32), vals=vals.astype(np.float32),
                         grid=wl.pixel_grid(side, side + q), basis=basis, precision=prec,
                         weight=weight, h=h))
    return reqs


def test_served_equals_direct(torch_dev):
    import torch
    from paper_1408_0677_amd import api
    reqs = make_requests()
    note(f"case server mix of {len(reqs)} requests on 4 slots")
    srv = api.Server(slots=4, hbm_budget=1 << 30, slot_scratch=64 << 20)
    tickets, outs = [], []
    for r in reqs:
        P = torch.from_numpy(r["pts"]).cuda()
        V = torch.from_numpy(r["vals"]).cuda()
        pid = srv.put_points(P, V)
        W, H = r["grid"]["width"], r["grid"]["height"]
        out = torch.full((V.shape[1], H, W), -7.0, device="cuda")
        deg = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
        t = srv.submit(pid, r["grid"], out, deg, basis=r["basis"], weight=r["weight"], h=r["h"],
                       precision=r["precision"])
        tickets.append(t)
        outs.append((out, deg, P, V))
    results = [srv.wait(t) for t in tickets]
    for r, res, (out, deg, P, V) in zip(reqs, results, outs):
        assert res["status"] == 0, res
        assert res["t_submit"] <= res["t_admit"] <= res["t_start"] <= res["t_end"]
        ref, rdeg = api.fit(P, V, r["grid"], basis=r["basis"], weight=r["weight"], h=r["h"],
                            precision=r["precision"])
        torch.cuda.synchronize()
        assert torch.equal(deg, rdeg)
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), r["precision"]
    srv.close()


def test_alone_vs_mix(torch_dev):
    """One request served alone on a one-slot server and inside a busy mix
    on a four-slot server gives identical bits."""
    import torch
    from paper_1408_0677_amd import api
    reqs = make_requests(seed=1, count=9)
    probe = reqs[4]
    note("case alone vs mix")

    def serve(slots, with_mix):
        srv = api.Server(slots=slots, hbm_budget=1 << 30, slot_scratch=64 << 20)
        keep = []
        todo = (reqs if with_mix else []) + [probe] + (reqs if with_mix else [])
        probe_out = None
        tickets = []
        for r in todo:
            P = torch.from_numpy(r["pts"]).cuda()
            V = torch.from_numpy(r["vals"]).cuda()
            pid = srv.put_points(P, V)
            W, H = r["grid"]["width"], r["grid"]["height"]
            out = torch.empty((V.shape[1], H, W), device="cuda")
            t = srv.submit(pid, r["grid"], out, None, basis=r["basis"], weight=r["weight"],
                           h=r["h"], precision=r["precision"])
            tickets.append(t)
            keep.append(out)
            if r is probe and probe_out is None:
                probe_out = out
        for t in tickets:
            assert srv.wait(t)["status"] == 0
        srv.close()
        return probe_out.cpu().numpy()

    alone = serve(1, False)
    mixed = serve(4, True)
    assert np.array_equal(alone.view(np.uint32), mixed.view(np.uint32))


def test_errors_are_isolated(torch_dev):
    import torch
    from paper_1408_0677_amd import api
    note("case server errors")
    srv = api.Server(slots=2, hbm_budget=256 << 20, slot_scratch=1 << 20)
    P = torch.rand(500, 2, device="cuda")
    V = torch.rand(500, 3, device="cuda")
    pid = srv.put_points(P, V)
    grid = {"x0": 0.0, "y0": 0.0, "dx": 0.02, "dy": 0.02, "width": 40, "height": 40}
    out = torch.empty((3, 40, 40), device="cuda")
    # refused at submit with mls_fit's own status (unsupported with f64)
    with pytest.raises(api.ServerError) as ei:
        srv.submit(pid, grid, out, weight="wendland")
    assert ei.value.status == -7 and "weight kind" in str(ei.value)
    good = srv.submit(pid, grid, torch.empty((3, 40, 40), device="cuda"), h=0.1)
    assert srv.wait(good)["status"] == 0
    # a request whose staging scratch cannot fit a slot is refused at submit
    big = torch.rand(200_000, 2, device="cuda")
    bigv = torch.rand(200_000, 4, device="cuda")
    pid2 = srv.put_points(big, bigv)
    with pytest.raises(api.ServerError) as ei:
        srv.submit(pid2, grid, torch.empty((4, 40, 40), device="cuda"), precision="bf16", h=0.1)
    assert "OVER_BUDGET" in str(ei.value)
    # a point set larger than the budget is refused
    with pytest.raises(api.ServerError):
        srv.put_points(torch.rand(30_000_000, 2, device="cuda"),
                       torch.rand(30_000_000, 1, device="cuda"))
    srv.release_points(pid)
    with pytest.raises(api.ServerError):
        srv.submit(pid, grid, out)
    srv.close()


def test_tuned_server_equals_direct(torch_dev, tmp_path):
    """With the autotuner on, the first request of each shape class is timed
    over candidate slab widths; every result still equals the direct fit
    bit for bit, and the chosen widths persist in the cache file."""
    import torch
    from paper_1408_0677_amd import api, workloads as wl
    note("case tuned server")
    cache = tmp_path / "tuner.txt"
    srv = api.Server(slots=3, hbm_budget=1 << 30, slot_scratch=64 << 20, tune=True,
                     tuner_cache=str(cache))
    rng = np.random.default_rng(5)
    reqs = []
    for q in range(8):
        n = 3000
        D = (24, 6)[q % 2]
        basis = ("quadratic", "linear")[q % 2]
        prec = ("bf16", "fp16")[(q // 2) % 2]
        pts = rng.random((n, 2)).astype(np.float32)
        vals = wl.smooth_fields(rng, pts, D).astype(np.float32)
        reqs.append((pts, vals, basis, prec))
    tickets, outs = [], []
    grid = wl.pixel_grid(128, 96)
    for pts, vals, basis, prec in reqs:
        P = torch.from_numpy(pts).cuda()
        V = torch.from_numpy(vals).cuda()
        pid = srv.put_points(P, V)
        out = torch.empty((V.shape[1], 96, 128), device="cuda")
        deg = torch.empty((96, 128), dtype=torch.uint8, device="cuda")
        tickets.append(srv.submit(pid, grid, out, deg, basis=basis, h=0.07, precision=prec))
        outs.append((out, deg, P, V, basis, prec))
    for t in tickets:
        assert srv.wait(t)["status"] == 0
    # the tuner runs beside the scheduler: wait for it to finish its classes
    t_end = time.time() + 60
    while srv.tuning_pending() and time.time() < t_end:
        time.sleep(0.01)
    assert srv.tuning_pending() == 0
    classes = srv.tuned_classes()
    assert classes == 4          # {bf16, fp16} x {quadratic D 24, linear D 6}
    for out, deg, P, V, basis, prec in outs:
        f, d = api.fit(P, V, grid, basis=basis, h=0.07, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(d, deg)
        assert torch.equal(f.view(torch.int32), out.view(torch.int32))
    srv.close()
    lines = [ln for ln in cache.read_text().splitlines() if "=" in ln]
    assert len(lines) == classes
    srv2 = api.Server(slots=1, hbm_budget=1 << 28, slot_scratch=16 << 20, tune=True,
                      tuner_cache=str(cache))
    assert srv2.tuned_classes() == classes
    srv2.close()


def class_requests(rng, count, grid_side=96):
    """16-bit Gaussian requests of a few kernel classes (bases, formats and
    attribute counts), small enough to share batches."""
    from paper_1408_0677_amd import workloads as wl
    reqs = []
    for q in range(count):
        n = int(rng.integers(300, 3000))
        d = int(rng.choice([3, 8, 13]))
        basis = ("linear", "quadratic")[q % 2]
        prec = ("fp16", "bf16")[(q // 2) % 2]
        pts = rng.random((n, 2)).astype(np.float32)
        vals = wl.smooth_fields(rng, pts, d).astype(np.float32)
        side = grid_side + int(rng.integers(0, 40))
        reqs.append(dict(pts=pts, vals=vals, basis=basis, precision=prec,
                         h=float(np.sqrt(40.0 / (np.pi * n))),
                         grid=wl.pixel_grid(side, side - 7)))
    return reqs


def submit_all(srv, reqs, **kw):
    import torch
    out = []
    for r in reqs:
        P = torch.from_numpy(r["pts"]).cuda()
        V = torch.from_numpy(r["vals"]).cuda()
        pid = srv.put_points(P, V)
        W, H = r["grid"]["width"], r["grid"]["height"]
        f = torch.full((V.shape[1], H, W), -3.0, device="cuda")
        g = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
        t = srv.submit(pid, r["grid"], f, g, basis=r["basis"], h=r["h"],
                       precision=r["precision"], **kw)
        out.append((t, f, g, P, V))
    return out


def test_batched_requests_equal_direct(torch_dev):
    """Many 16-bit requests submitted at once to a one-slot server run as a
    few persistent batches (members of a batch share their start time);
    every request equals its direct mls_fit bit for bit."""
    import torch
    from paper_1408_0677_amd import api
    rng = np.random.default_rng(11)
    reqs = class_requests(rng, 24)
    note(f"case batched server: {len(reqs)} requests, 1 slot")
    srv = api.Server(slots=1, hbm_budget=1 << 30, slot_scratch=128 << 20)
    subs = submit_all(srv, reqs)
    results = [srv.wait(t) for t, *_ in subs]
    starts = set()
    for r, res, (t, f, g, P, V) in zip(reqs, results, subs):
        assert res["status"] == 0, res
        assert res["t_submit"] <= res["t_admit"] <= res["t_start"] <= res["t_end"]
        starts.add(res["t_start"])
        ref, rdeg = api.fit(P, V, r["grid"], basis=r["basis"], h=r["h"],
                            precision=r["precision"])
        torch.cuda.synchronize()
        assert torch.equal(g, rdeg)
        assert torch.equal(f.view(torch.int32), ref.view(torch.int32)), r
    note(f"  {len(starts)} launches for {len(reqs)} requests")
    assert len(starts) < len(reqs)
    srv.close()


def test_cancel_and_timeout_in_the_queue(torch_dev):
    """Behind a long float64 request on a one-slot server: a cancelled
    queued request and one whose timeout passes in the queue end with
    MLS_ERR_CANCELLED and leave their outputs untouched; the others finish
    and equal their direct fits."""
    import torch
    from paper_1408_0677_amd import api, workloads as wl
    note("case cancel and timeout in the queue")
    rng = np.random.default_rng(12)
    srv = api.Server(slots=1, hbm_budget=1 << 30, slot_scratch=64 << 20)
    n = 40000
    P = torch.rand(n, 2, device="cuda")
    V = torch.rand(n, 4, device="cuda")
    pid = srv.put_points(P, V)
    big_grid = wl.pixel_grid(1024)
    big = torch.empty((4, 1024, 1024), device="cuda")
    t_big = srv.submit(pid, big_grid, big, basis="quadratic", h=0.02, precision="f64")
    reqs = class_requests(rng, 3)
    subs = submit_all(srv, reqs[:2])
    subs += submit_all(srv, reqs[2:], timeout_s=1e-4)
    srv.cancel(subs[1][0])
    res = [srv.wait(t) for t, *_ in subs]
    assert srv.wait(t_big)["status"] == 0
    assert res[0]["status"] == 0
    assert res[1]["status"] == -6 and "queue" in res[1]["detail"], res[1]
    assert res[2]["status"] == -6 and "timeout" in res[2]["detail"], res[2]
    for k in (1, 2):
        assert bool((subs[k][1] == -3.0).all())
    r, (t, f, g, P0, V0) = reqs[0], subs[0]
    ref, _ = api.fit(P0, V0, r["grid"], basis=r["basis"], h=r["h"], precision=r["precision"])
    torch.cuda.synchronize()
    assert torch.equal(f.view(torch.int32), ref.view(torch.int32))
    # a finished (collected) ticket can no longer be cancelled
    with pytest.raises(api.ServerError):
        srv.cancel(subs[0][0])
    srv.close()


def test_timeout_inside_a_running_batch(torch_dev):
    """A large batched request whose timeout passes while its kernel runs
    has its remaining work items skipped (MLS_ERR_CANCELLED); the server
    then serves the next request of the same class correctly."""
    import torch
    from paper_1408_0677_amd import api, workloads as wl
    note("case timeout inside a running batch")
    rng = np.random.default_rng(13)
    srv = api.Server(slots=1, hbm_budget=4 << 30, slot_scratch=64 << 20)
    n, d = 20000, 32
    pts = rng.random((n, 2)).astype(np.float32)
    vals = wl.smooth_fields(rng, pts, d).astype(np.float32)
    P = torch.from_numpy(pts).cuda()
    V = torch.from_numpy(vals).cuda()
    pid = srv.put_points(P, V)
    h = float(np.sqrt(40.0 / (np.pi * n)))
    small = wl.pixel_grid(384)
    # load the class's kernel first
    warm = torch.empty((d, 384, 384), device="cuda")
    assert srv.wait(srv.submit(pid, small, warm, basis="quadratic", h=h,
                               precision="fp16"))["status"] == 0
    grid = wl.pixel_grid(2048)
    out = torch.empty((d, 2048, 2048), device="cuda")
    t = srv.submit(pid, grid, out, basis="quadratic", h=h, precision="fp16", timeout_s=0.004)
    res = srv.wait(t)
    note(f"  status {res['status']} after {1e3 * (res['t_end'] - res['t_submit']):.1f} ms: "
         f"{res['detail']}")
    assert res["status"] == -6 and "skipped" in res["detail"], res
    assert res["t_end"] - res["t_submit"] < 1.0
    # the slot is reused by the next batch: flags and counters start clean
    again = torch.empty((d, 384, 384), device="cuda")
    assert srv.wait(srv.submit(pid, small, again, basis="quadratic", h=h,
                               precision="fp16"))["status"] == 0
    torch.cuda.synchronize()
    assert torch.equal(again.view(torch.int32), warm.view(torch.int32))
    srv.close()
