"""Serving loop over the library's continuous-batching server (gdn_server_*).

``Server`` wraps one gdn_server; ``simulate`` streams frames from simulated
sensors (Poisson arrivals) into it in real time, polls it, and reports
per-frame latency (arrival to completion seen by the poll) and throughput.
Frames may sit on the device or arrive in pinned host memory (copied to the
device on a copy stream first); every request gets its own output buffers.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as B


class Server:
    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_slots: int = 4,
                 slot_points: int = 1 << 20, slot_frames: int = 16, **params):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.srv = 0
        self.flagged = {}
        self.ctx = B.gdn_create(device)
        self.params = B.make_params(**params)
        try:
            self.srv = B.gdn_server_create(self.ctx, self.params, hbm_budget, max_slots, slot_points, slot_frames)
        except Exception:
            self.close()
            raise
        self.n_slots, self.bytes_per_slot = B.gdn_server_info(self.srv)
        self.slot_points = slot_points

    def close(self):
        if self.srv:
            B.gdn_server_destroy(self.srv)
            self.srv = 0
        if self.ctx:
            B.gdn_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc(self, n: int) -> B.Result:
        t = self.torch
        d = self.device
        return B.Result(keep=t.empty(n, dtype=t.uint8, device=d), score=t.empty(n, dtype=t.float32, device=d),
                        stage=t.empty(n, dtype=t.uint8, device=d), kept_idx=t.empty(n, dtype=t.int32, device=d),
                        n_kept=t.empty(1, dtype=t.int64, device=d))

    def submit(self, xyz, out: B.Result) -> int:
        n = xyz.shape[0]
        return B.gdn_server_submit(self.srv, xyz.data_ptr(), n, out.keep.data_ptr(), out.score.data_ptr(),
                                   out.stage.data_ptr(), out.kept_idx.data_ptr(), out.n_kept.data_ptr())

    def poll(self):
        """(finished tickets, queue length, busy slots). Raises GdnError if a
        finished frame's batch raised a device status bit (its outputs are
        unspecified); the tickets of such a batch are in ``self.flagged``."""
        done, sts, nw, nb = B.gdn_server_poll(self.srv)
        bad = {t: s for t, s in zip(done, sts) if s}
        if bad:
            self.flagged.update(bad)
            raise B.GdnError(B.GDN_EINTERNAL, f"device status {sorted(set(bad.values()))} for tickets {sorted(bad)}")
        return done, nw, nb


def arrivals(n_sensors: int, rate_hz: float, duration_s: float, seed: int):
    """Merged Poisson arrival times of n_sensors sensors: [(t, sensor)]."""
    rng = np.random.default_rng(seed)
    ev = []
    for s in range(n_sensors):
        t = rng.exponential(1.0 / rate_hz)
        while t < duration_s:
            ev.append((t, s))
            t += rng.exponential(1.0 / rate_hz)
    ev.sort()
    return ev


def simulate(server: Server, frames, n_sensors: int = 16, rate_hz: float = 10.0, duration_s: float = 32.0,
             warmup_s: float = 2.0, seed: int = 5, log=None):
    """Stream frames (picked round-robin per sensor) into the server at their
    Poisson arrival times; returns latency percentiles and throughput over the
    arrivals after the warm-up.

    Frames on the device are submitted as they arrive. Frames in (pinned)
    host memory are first copied to the device on a copy stream; each is
    submitted once its copy has completed, so its latency includes the copy."""
    torch = server.torch
    ev = arrivals(n_sensors, rate_hz, duration_s, seed)
    host = frames[0].device.type == "cpu"
    copy_stream = torch.cuda.Stream(device=server.device) if host else None
    copying = []   # (event, device tensor, arrival time) in arrival order
    torch.cuda.synchronize()  # the frames are written before the server's streams read them
    outs = {}
    pending = {}   # ticket -> (arrival wall time, n points, sensor seq)
    lat, pts_done, lat_pts = [], 0, 0
    t0 = time.perf_counter()
    i = 0
    seq = [0] * n_sensors
    last_log = t0

    def submit(x, t_arr):
        out = server.alloc(x.shape[0])
        tk = server.submit(x, out)
        outs[tk] = (out, x)
        pending[tk] = (t_arr, x.shape[0])

    while i < len(ev) or pending or copying:
        now = time.perf_counter() - t0
        while i < len(ev) and ev[i][0] <= now:
            t_arr, s = ev[i]
            f = frames[(s * 7 + seq[s]) % len(frames)]
            seq[s] += 1
            if host:
                with torch.cuda.stream(copy_stream):
                    d = torch.empty(f.shape, dtype=f.dtype, device=server.device)
                    d.copy_(f, non_blocking=True)
                    e = torch.cuda.Event()
                    e.record(copy_stream)
                copying.append((e, d, t_arr))
            else:
                submit(f, t_arr)
            i += 1
        while copying and copying[0][0].query():
            _, d, t_arr = copying.pop(0)
            submit(d, t_arr)
        done, nw, nb = server.poll()
        now = time.perf_counter() - t0
        for tk in done:
            t_arr, n = pending.pop(tk)
            outs.pop(tk)
            if t_arr >= warmup_s:
                lat.append((now - t_arr) * 1e3)
                lat_pts += n
        if not done and not copying and (i >= len(ev) or ev[i][0] > now):
            time.sleep(0.0001)
        if log and now - (last_log - t0) > 5.0:
            last_log = time.perf_counter()
            log(f"[serve] t={now:.1f}s submitted={i} in-flight={len(pending)} waiting={nw} busy={nb}")
    torch.cuda.synchronize()
    window = duration_s - warmup_s
    lat = np.array(lat)
    return {"frames": int(len(lat)), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "mpoints_s": lat_pts / window / 1e6,
            "offered_frames_s": n_sensors * rate_hz, "window_s": window, "slots": server.n_slots,
            "bytes_per_slot": server.bytes_per_slot}
