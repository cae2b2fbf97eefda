"""Seeded synthetic point-cloud frames.

This module only draws inputs: coordinates and ground-truth noise labels. It
holds none of the denoiser's arithmetic, so both the CPU oracle (through the
tests) and the HIP path can be fed from it.

The paper evaluates on the Stanford Bunny with injected random noise (Sec. 4.1,
Table 1), a CADC snow frame (Sec. 4.2.3) and in-house FMCW LiDAR frames
(Sec. 4.2.4). None of those datasets is available here; the generators below
stand in for them with the same kinds of geometry, sizes and noise mixes:

* ``sphere_plane``: a scanned-object-like cloud (surfaces + uniform outliers),
  the stand-in for the Bunny-with-random-noise frames.
* ``lidar_frame``: a spinning 64-beam LiDAR frame over a ground plane, boxes and
  a far wall, with near-sensor snow returns, the stand-in for the CADC snow
  frame and the 50 m / 100 m FMCW frames (about 120k points).
* ``torus_bumpy``: a torus and a bumpy sphere with Gaussian surface noise at a
  given fraction of the bounding-box diagonal plus 10% uniform outliers, the
  stand-in for the Bunny frames at several noise levels (score-fit sets).

Every frame is returned as ``(xyz float32 [N,3], label uint8 [N])`` with
label 1 marking an injected noise point. Rows are shuffled with a seeded
permutation so that input order carries no spatial structure.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "sphere_plane",
    "lidar_frame",
    "lidar_batch_sizes",
    "uniform_cube",
    "torus_bumpy",
    "fit_set",
    "CONFIGS",
]


def _shuffle(rng, xyz, label):
    perm = rng.permutation(xyz.shape[0])
    return (np.ascontiguousarray(xyz[perm], dtype=np.float32),
            np.ascontiguousarray(label[perm], dtype=np.uint8))


def sphere_plane(seed: int = 1, n_sphere: int = 12137, n_plane: int = 3863,
                 n_out: int = 4000, sigma: float = 0.005):
    """Unit sphere + z=0 square plane + uniform outliers (20,000 points).

    The surface split 12,137 : 3,863 is area-proportional (4*pi : 4). The plane
    cuts the sphere at its equator, which gives sharp edges. Every surface point
    gets isotropic Gaussian jitter of std ``sigma``; outliers are uniform in the
    cube [-1.5, 1.5]^3 and carry label 1.
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n_sphere, 3))
    sph = g / np.linalg.norm(g, axis=1, keepdims=True)
    pl = np.column_stack([rng.uniform(-1.0, 1.0, n_plane),
                          rng.uniform(-1.0, 1.0, n_plane),
                          np.zeros(n_plane)])
    surf = np.concatenate([sph, pl], axis=0)
    surf = surf + rng.normal(0.0, sigma, surf.shape)
    out = rng.uniform(-1.5, 1.5, (n_out, 3))
    xyz = np.concatenate([surf, out], axis=0).astype(np.float32)
    label = np.concatenate([np.zeros(surf.shape[0], np.uint8),
                            np.ones(n_out, np.uint8)])
    return _shuffle(rng, xyz, label)


def uniform_cube(seed: int, n: int, side: float = 1.0):
    """n points uniform in [0, side)^3 (label 0). Small test clouds."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(0.0, side, (n, 3)).astype(np.float32)
    return xyz, np.zeros(n, np.uint8)


def torus_bumpy(seed: int = 30, noise_frac: float = 0.01, n_torus: int = 90_000, n_bumpy: int = 90_000,
                n_out: int = 20_000):
    """Torus (R = 1, r = 0.35, axis z, at the origin) + bumpy sphere
    r(theta, phi) = 0.8 (1 + 0.1 sin(6 theta) cos(6 phi)) centred at (2.6, 0, 0),
    both sampled close to area-uniform by rejection (torus: weight
    (R + r cos v) / (R + r); sphere: weight r^2 / r_max^2, the slope of the
    bumps ignored). Surface points get isotropic Gaussian noise of std
    ``noise_frac`` x the clean bounding-box diagonal; ``n_out`` outliers
    (label 1) are uniform in the clean box grown by 10% about its centre.
    """
    rng = np.random.default_rng(seed)
    R, r = 1.0, 0.35
    tor = np.zeros((0, 3))
    while tor.shape[0] < n_torus:
        m = 2 * (n_torus - tor.shape[0]) + 64
        u = rng.uniform(0.0, 2 * np.pi, m)
        v = rng.uniform(0.0, 2 * np.pi, m)
        ok = rng.uniform(0.0, 1.0, m) < (R + r * np.cos(v)) / (R + r)
        u, v = u[ok], v[ok]
        pts = np.column_stack([(R + r * np.cos(v)) * np.cos(u), (R + r * np.cos(v)) * np.sin(u), r * np.sin(v)])
        tor = np.concatenate([tor, pts])
    tor = tor[:n_torus]
    bum = np.zeros((0, 3))
    rmax = 0.8 * 1.1
    while bum.shape[0] < n_bumpy:
        m = 2 * (n_bumpy - bum.shape[0]) + 64
        g = rng.standard_normal((m, 3))
        d = g / np.linalg.norm(g, axis=1, keepdims=True)
        th = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
        ph = np.arctan2(d[:, 1], d[:, 0])
        rr = 0.8 * (1.0 + 0.1 * np.sin(6 * th) * np.cos(6 * ph))
        ok = rng.uniform(0.0, 1.0, m) < (rr / rmax) ** 2
        bum = np.concatenate([bum, d[ok] * rr[ok, None] + np.array([2.6, 0.0, 0.0])])
    bum = bum[:n_bumpy]
    surf = np.concatenate([tor, bum])
    lo, hi = surf.min(0), surf.max(0)
    diag = float(np.linalg.norm(hi - lo))
    surf = surf + rng.normal(0.0, noise_frac * diag, surf.shape)
    c, h = (lo + hi) / 2, (hi - lo) / 2 * 1.1
    out = rng.uniform(c - h, c + h, (n_out, 3))
    xyz = np.concatenate([surf, out]).astype(np.float32)
    label = np.concatenate([np.zeros(surf.shape[0], np.uint8), np.ones(n_out, np.uint8)])
    return _shuffle(rng, xyz, label)


FIT_NOISE = (0.005, 0.01, 0.02)


def fit_set(seed: int = 30, n_torus: int = 90_000, n_bumpy: int = 90_000, n_out: int = 20_000):
    """Score-fit frames: ``torus_bumpy`` at the noise levels FIT_NOISE, scene
    seeds seed, seed + 1, seed + 2. Returns (list of xyz, list of labels)."""
    fr = [torus_bumpy(seed + i, f, n_torus, n_bumpy, n_out) for i, f in enumerate(FIT_NOISE)]
    return [x for x, _ in fr], [lab for _, lab in fr]


# ---------------------------------------------------------------------------
# LiDAR-like frame
# ---------------------------------------------------------------------------

_SENSOR = np.array([0.0, 0.0, 1.8])
_WALL_R = 80.0
_WALL_H = 12.0


def _scene_boxes(rng):
    """12 axis-aligned boxes standing on the ground: 9 car-like, 3 buildings."""
    boxes = []
    for i in range(12):
        building = i >= 9
        if building:
            sx, sy, sz = rng.uniform(10.0, 20.0, 3)
            dist = rng.uniform(35.0, 60.0)
        else:
            sx = rng.uniform(3.5, 4.8)
            sy = rng.uniform(1.6, 2.0)
            sz = rng.uniform(1.4, 1.8)
            dist = rng.uniform(4.0 + 3.0, 40.0)
        az = rng.uniform(0.0, 2.0 * np.pi)
        cx, cy = dist * np.cos(az), dist * np.sin(az)
        lo = np.array([cx - sx / 2, cy - sy / 2, 0.0])
        hi = np.array([cx + sx / 2, cy + sy / 2, sz])
        boxes.append((lo, hi))
    return boxes


def _first_hit(dirs, boxes):
    """Range along each unit ray from the sensor to the first surface."""
    n = dirs.shape[0]
    t = np.full(n, np.inf)
    # ground plane z = 0
    dz = dirs[:, 2]
    down = dz < 0
    tg = np.where(down, -_SENSOR[2] / np.where(down, dz, -1.0), np.inf)
    t = np.minimum(t, tg)
    # cylindrical wall x^2 + y^2 = R^2, 0 <= z <= H
    dxy = np.hypot(dirs[:, 0], dirs[:, 1])
    tw = np.where(dxy > 0, _WALL_R / np.where(dxy > 0, dxy, 1.0), np.inf)
    zw = _SENSOR[2] + tw * dz
    tw = np.where((zw >= 0.0) & (zw <= _WALL_H), tw, np.inf)
    t = np.minimum(t, tw)
    # boxes (slab test)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dirs
        for lo, hi in boxes:
            t0 = (lo - _SENSOR) * inv
            t1 = (hi - _SENSOR) * inv
            tmin = np.nanmax(np.minimum(t0, t1), axis=1)
            tmax = np.nanmin(np.maximum(t0, t1), axis=1)
            hit = (tmax >= np.maximum(tmin, 0.0)) & (tmin > 0)
            t = np.where(hit & (tmin < t), tmin, t)
    return t


def lidar_frame(seed: int = 2, n_beams: int = 64, n_az: int = 1875,
                range_sigma: float = 0.02, snow_frac: float = 0.05,
                el_top_deg: float = 2.0, el_bot_deg: float = -24.8):
    """Spinning LiDAR frame of ``n_beams * n_az`` points.

    Sensor at (0, 0, 1.8) m; beam elevations evenly spaced from +2.0 deg to
    -24.8 deg; ``n_az`` azimuth steps over 360 deg. The scene is the ground
    plane, 9 car-sized and 3 building-sized boxes, and a 12 m wall at 80 m
    radius. Measured range = first-hit range clipped to [2, 80] m plus
    N(0, range_sigma^2) along the ray. A seeded ``snow_frac`` of the rays are
    replaced by snow returns at a range drawn uniformly in
    [2, min(15, true range)] m; those carry label 1.
    """
    rng = np.random.default_rng(seed)
    boxes = _scene_boxes(rng)
    el = np.deg2rad(np.linspace(el_top_deg, el_bot_deg, n_beams))
    az = np.arange(n_az) * (2.0 * np.pi / n_az)
    az = az + rng.uniform(0.0, 2.0 * np.pi / n_az)  # random phase of the sweep
    E, A = np.meshgrid(el, az, indexing="ij")
    dirs = np.column_stack([(np.cos(E) * np.cos(A)).ravel(),
                            (np.cos(E) * np.sin(A)).ravel(),
                            np.sin(E).ravel()])
    n = dirs.shape[0]
    t_true = _first_hit(dirs, boxes)
    r = np.clip(t_true, 2.0, 80.0) + rng.normal(0.0, range_sigma, n)
    label = np.zeros(n, np.uint8)
    n_snow = int(round(snow_frac * n))
    snow = rng.choice(n, size=n_snow, replace=False)
    hi = np.minimum(15.0, np.clip(t_true[snow], 2.0, 80.0))
    r[snow] = rng.uniform(2.0, hi)
    label[snow] = 1
    xyz = (_SENSOR[None, :] + r[:, None] * dirs).astype(np.float32)
    return _shuffle(rng, xyz, label)


def lidar_batch_sizes(seed: int = 4000, n_frames: int = 64,
                      lo: int = 60_000, hi: int = 130_000, n_beams: int = 64):
    """Azimuth step counts for a batch of uneven LiDAR frames.

    Frame sizes are drawn uniformly in [lo, hi] and rounded to a whole number
    of azimuth steps, so each frame has ``n_beams * n_az`` points.
    """
    rng = np.random.default_rng(seed)
    sizes = rng.uniform(lo, hi, n_frames)
    return [int(round(s / n_beams)) for s in sizes]


def lidar_batch(seed: int = 4000, n_frames: int = 64, lo: int = 60_000, hi: int = 130_000):
    """Uneven LiDAR frames for batched runs: frame f has the azimuth count
    ``lidar_batch_sizes(seed, n_frames, lo, hi)[f]`` and scene seed ``seed + f``.
    Returns (list of xyz arrays, list of label arrays)."""
    sizes = lidar_batch_sizes(seed, n_frames, lo, hi)
    out = [lidar_frame(seed=seed + f, n_az=s) for f, s in enumerate(sizes)]
    return [x for x, _ in out], [lab for _, lab in out]


# Workload recipes: generator, its arguments and the method parameters they
# are run with. Parameters not named here take the library defaults.
CONFIGS = {
    "sphere_plane_20k": dict(gen="sphere_plane", kwargs=dict(seed=1),
                             params=dict(k=16, leaf_cap=512)),
    "lidar_120k": dict(gen="lidar_frame", kwargs=dict(seed=2),
                       params=dict(k=32, leaf_cap=1024)),
    # 64 frames of 60k-130k points (6.2M in all); the leaf cap is autotuned
    # over LIDAR_BATCH_CAPS, 1024 is the starting value
    "lidar_batch_64": dict(gen="lidar_batch", kwargs=dict(seed=4000, n_frames=64),
                           params=dict(k=32, leaf_cap=1024)),
    # frame pool of a served stream: 32 LiDAR frames of 20k-130k points that
    # simulated sensors send round-robin; leaf cap 256, the autotuner's choice
    # for batches of this generator's frames (listed after the fit set)
    # three 200k-point score-fit frames (noise 0.5%, 1%, 2% of the diagonal)
    "fit_200k": dict(gen="fit_set", kwargs=dict(seed=30), params=dict(k=16, leaf_cap=512)),
    "lidar_stream_pool": dict(gen="lidar_batch", kwargs=dict(seed=5000, n_frames=32, lo=20_000, hi=130_000),
                              params=dict(k=32, leaf_cap=256)),
}

LIDAR_BATCH_CAPS = (256, 512, 1024, 2048)


def make(name: str):
    """Return (xyz, label, params) for a named workload recipe (for a batch,
    xyz and label are lists with one array per frame)."""
    c = CONFIGS[name]
    fn = {"sphere_plane": sphere_plane, "lidar_frame": lidar_frame, "lidar_batch": lidar_batch,
          "fit_set": fit_set}[c["gen"]]
    xyz, label = fn(**c["kwargs"])
    return xyz, label, dict(c["params"])
