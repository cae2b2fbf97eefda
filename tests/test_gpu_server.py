"""Continuous-batching server (gdn_server_*) through the C ABI.

A served frame shares its slot's batch with whatever other frames were
waiting, so the test is that each frame's results are the ones it gets when
denoised alone (gdn_denoise), bit for bit, whatever the mix: the batched path
runs every frame on its own (its own box, octree and percentiles), and the
plain path is checked against the oracle in test_gpu_parity.py.
"""
import time

import numpy as np
import pytest

from paper_2512_10386_amd import synth

pytestmark = pytest.mark.gpu

PARAMS = dict(k=32, leaf_cap=512)


def server_frames():
    """Uneven frames: LiDAR sweeps of 2.5k-20k points, a scanned object, tiny ones."""
    fr = [synth.lidar_frame(seed=100 + i, n_az=a)[0]
          for i, a in enumerate([120, 300, 40, 200, 90, 250, 60, 150, 310, 70, 180, 100])]
    fr.insert(5, synth.sphere_plane(seed=9, n_sphere=6000, n_plane=2000, n_out=1500)[0])
    fr.insert(3, synth.uniform_cube(7, 1)[0])
    fr.insert(9, synth.uniform_cube(8, 33)[0])
    return [np.ascontiguousarray(f, np.float32) for f in fr]


def host(res, n):
    nk = int(res.n_kept.cpu().numpy()[0])
    return dict(keep=res.keep.cpu().numpy()[:n], score=res.score.cpu().numpy()[:n],
                stage=res.stage.cpu().numpy()[:n], n_kept=nk,
                kept=res.kept_idx.cpu().numpy().view(np.uint32)[:nk].copy())


@pytest.fixture(scope="module")
def frames():
    import torch
    fr = server_frames()
    return fr, [torch.from_numpy(f).cuda() for f in fr]


@pytest.fixture(scope="module")
def alone(frames):
    import torch
    from paper_2512_10386_amd.binding import Denoiser
    d = Denoiser(0, **PARAMS)
    out = []
    for x in frames[1]:
        out.append(host(d(x), x.shape[0]))
    torch.cuda.synchronize()
    d.close()
    return out


def serve(srv, devs, order, burst):
    """Submit frames in `order`, `burst` at a time with a poll between bursts;
    poll until all are done. Returns {frame: host results}."""
    import torch
    torch.cuda.synchronize()  # inputs written before the server's streams read them
    outs, ticket_of, done = {}, {}, set()
    t0 = time.time()
    pos = 0
    while len(done) < len(order):
        assert time.time() - t0 < 60.0, "server did not finish"
        for f in order[pos:pos + burst]:
            o = srv.alloc(devs[f].shape[0])
            ticket_of[srv.submit(devs[f], o)] = f
            outs[f] = o
        pos += burst
        fin, _, _ = srv.poll()
        done.update(fin)
        if pos >= len(order) and not fin:
            time.sleep(0.001)
    torch.cuda.synchronize()
    return {ticket_of[t]: host(outs[ticket_of[t]], devs[ticket_of[t]].shape[0]) for t in done}


def check_same(got, ref, f):
    for key in ("keep", "score", "stage"):
        assert np.array_equal(got[key].view(np.uint8), ref[key].view(np.uint8)), (f, key)
    assert got["n_kept"] == ref["n_kept"], f
    assert np.array_equal(got["kept"], ref["kept"]), f


@pytest.mark.parametrize("order_kind,burst,slots", [("fifo", 100, 3), ("reverse", 2, 2), ("shuffled", 3, 4)])
def test_served_frames_equal_alone(frames, alone, order_kind, burst, slots):
    from paper_2512_10386_amd.serve import Server
    nf = len(frames[0])
    order = list(range(nf))
    if order_kind == "reverse":
        order = order[::-1]
    elif order_kind == "shuffled":
        order = list(np.random.default_rng(3).permutation(nf))
    srv = Server(0, hbm_budget=8 << 30, max_slots=slots, slot_points=40_000, slot_frames=3, **PARAMS)
    try:
        assert srv.n_slots == slots
        got = serve(srv, frames[1], order, burst)
    finally:
        srv.close()
    assert sorted(got) == list(range(nf))
    for f in range(nf):
        check_same(got[f], alone[f], f)


def test_server_reuses_slots_over_many_requests(frames, alone):
    """Every frame three times through one slot of two frames: slots and their
    workspaces are reused with different mixes each time."""
    from paper_2512_10386_amd.serve import Server
    nf = len(frames[0])
    srv = Server(0, hbm_budget=8 << 30, max_slots=1, slot_points=25_000, slot_frames=2, **PARAMS)
    try:
        for rep in range(3):
            order = list(np.random.default_rng(10 + rep).permutation(nf))
            got = serve(srv, frames[1], order, 4)
            for f in range(nf):
                check_same(got[f], alone[f], f)
    finally:
        srv.close()


def test_served_configuration_equals_alone():
    """The served workload as the benchmark runs it: LiDAR frames of 20k-130k
    points from the stream pool, k = 32, leaf cap 256, the benchmark's slot
    shape (4 Mi points, 64 frames: a slot filled from the burst exceeds 2^20
    points and runs the large-input kernels, while each frame alone runs the
    small-input ones). Every served frame equals the same frame denoised
    alone, bit for bit, and no batch raised a device status bit."""
    import torch
    from paper_2512_10386_amd.binding import Denoiser
    from paper_2512_10386_amd.serve import Server
    pool, _, params = synth.make("lidar_stream_pool")
    assert params == dict(k=32, leaf_cap=256)
    devs = [torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in pool]
    d = Denoiser(0, **params)
    alone = [host(d(x), x.shape[0]) for x in devs]
    torch.cuda.synchronize()
    d.close()
    order = list(np.random.default_rng(55).permutation(len(devs))) * 2  # every frame twice, 64 requests
    from bench import SERVE_SLOT_FRAMES, SERVE_SLOT_POINTS
    srv = Server(0, hbm_budget=32 << 30, max_slots=4, slot_points=SERVE_SLOT_POINTS, slot_frames=SERVE_SLOT_FRAMES,
                 **params)
    try:
        got = serve_tickets(srv, devs, order, 64)
    finally:
        srv.close()
    assert srv.flagged == {}
    assert len(got) == len(order)
    for f, res in got:
        check_same(res, alone[f], f)
    # the first slot packed from the burst crosses 2^20 points
    tot, first = 0, 0
    for f in order[:SERVE_SLOT_FRAMES]:
        if tot + devs[f].shape[0] > SERVE_SLOT_POINTS:
            break
        tot += devs[f].shape[0]
        first += 1
    assert tot > (1 << 20), tot
    print(f"[serve] first batch {first} frames, {tot} points", flush=True)


def serve_tickets(srv, devs, order, burst):
    """Like serve(), but a frame may be submitted more than once: returns
    [(frame, host results)] per ticket."""
    import torch
    torch.cuda.synchronize()
    outs, ticket_of, done = {}, {}, []
    t0 = time.time()
    pos = 0
    while len(done) < len(order):
        assert time.time() - t0 < 60.0, "server did not finish"
        for f in order[pos:pos + burst]:
            o = srv.alloc(devs[f].shape[0])
            t = srv.submit(devs[f], o)
            ticket_of[t] = f
            outs[t] = o
        pos += burst
        fin, _, _ = srv.poll()
        done.extend(fin)
        if pos >= len(order) and not fin:
            time.sleep(0.001)
    torch.cuda.synchronize()
    return [(ticket_of[t], host(outs[t], devs[ticket_of[t]].shape[0])) for t in sorted(done)]


def test_server_errors(frames):
    import torch
    from paper_2512_10386_amd import binding as B
    from paper_2512_10386_amd.serve import Server
    srv = Server(0, hbm_budget=1 << 30, max_slots=2, slot_points=10_000, slot_frames=2, **PARAMS)
    try:
        _, per_slot = B.gdn_server_info(srv.srv)
        assert srv.n_slots == min(2, (1 << 30) // per_slot)
        big = torch.zeros((10_001, 3), dtype=torch.float32, device="cuda")
        with pytest.raises(B.GdnError) as e:
            srv.submit(big, srv.alloc(10_001))
        assert e.value.status == B.GDN_ECAPACITY
        empty = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
        with pytest.raises(B.GdnError) as e:
            srv.submit(empty, srv.alloc(1))
        assert e.value.status == B.GDN_EINVAL
        fin, nw, nb = srv.poll()
        assert fin == [] and nw == 0 and nb == 0
    finally:
        srv.close()
    with pytest.raises(B.GdnError) as e:
        Server(0, hbm_budget=1 << 20, max_slots=2, slot_points=100_000, slot_frames=4, **PARAMS)
    assert e.value.status == B.GDN_ENOMEM


@pytest.mark.parametrize("where", ["device", "host"])
def test_simulated_stream_runs(frames, where):
    """A short real-time run of the serving loop, frames on the device or in
    pinned host memory (copied on a copy stream first): every arrival is
    served."""
    from paper_2512_10386_amd.serve import Server, simulate
    src = frames[1] if where == "device" else [x.cpu().pin_memory() for x in frames[1]]
    srv = Server(0, hbm_budget=8 << 30, max_slots=3, slot_points=80_000, slot_frames=8, **PARAMS)
    try:
        r = simulate(srv, src, n_sensors=8, rate_hz=20.0, duration_s=1.5, warmup_s=0.5, seed=1)
    finally:
        srv.close()
    assert r["frames"] > 0 and r["p50_ms"] > 0 and r["p99_ms"] >= r["p50_ms"]
