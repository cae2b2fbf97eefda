"""Batched path (gdn_denoise_batch, graph replays, autotuner) through the C ABI.

A batch runs the method on every frame on its own, so each frame's outputs and
intermediates must equal those of a plain gdn_denoise call on that frame, bit
for bit (same keys, leaves, candidate sets and arithmetic). The plain path is
itself checked against the oracle in test_gpu_parity.py; one batch frame is
also checked against the oracle directly here.
"""
import numpy as np
import pytest

from paper_2512_10386_amd import synth
from tests.parity import compare, leaf_thresholds, run_gpu

pytestmark = pytest.mark.gpu

PER_POINT = ("KEYS", "OCC", "P1", "NBR_IDX", "NBR_D2", "R2K", "RHO", "P2", "SCORE64", "LEAF_OF", "ORDER")


@pytest.fixture(scope="module")
def bden():
    from paper_2512_10386_amd.binding import BatchDenoiser
    d = BatchDenoiser(0)
    yield d
    d.close()


@pytest.fixture(scope="module")
def den():
    from paper_2512_10386_amd.binding import Denoiser
    d = Denoiser(0)
    yield d
    d.close()


def frames_mixed():
    """Uneven frames: LiDAR, scanned object, uniform, tiny, single, empty."""
    fr = [synth.lidar_frame(seed=11, n_az=160)[0],
          synth.sphere_plane(seed=3, n_sphere=3000, n_plane=1000, n_out=800)[0],
          np.zeros((0, 3), np.float32),
          synth.uniform_cube(5, 2500)[0],
          synth.uniform_cube(6, 1)[0],
          synth.uniform_cube(7, 5)[0],
          synth.lidar_frame(seed=12, n_az=90)[0]]
    return [np.ascontiguousarray(f, np.float32) for f in fr]


def to_dev(frames):
    import torch
    off = np.zeros(len(frames) + 1, np.int64)
    off[1:] = np.cumsum([len(f) for f in frames])
    xyz = np.concatenate(frames) if off[-1] else np.zeros((0, 3), np.float32)
    return torch.from_numpy(xyz).cuda(), torch.from_numpy(off).cuda(), off


def batch_dumps(bden, n, nf):
    import torch
    torch.cuda.synchronize()
    d = {w: bden.dump(w, n).cpu().numpy() for w in PER_POINT}
    counts = bden.dump("COUNTS", n).cpu().numpy()
    d["n_leaves"] = int(counts[0])
    d["status"] = int(bden.dump("STATUS", n).cpu().numpy()[0])
    lt = bden.dump("LEAF_TABLE", n).cpu().numpy().view(np.uint32)[:d["n_leaves"]]
    d["LEAF_TABLE"] = lt
    return d


def outputs(res, n, nf):
    import torch
    torch.cuda.synchronize()
    return dict(keep=res.keep.cpu().numpy()[:n], score=res.score.cpu().numpy()[:n],
                stage=res.stage.cpu().numpy()[:n], kept_idx=res.kept_idx.cpu().numpy().view(np.uint32)[:n],
                n_kept=res.n_kept.cpu().numpy()[:nf])


def kept_lists(o, off):
    """Per-frame kept indices (entries past a frame's count are unspecified)."""
    return [o["kept_idx"][int(off[f]):int(off[f]) + int(o["n_kept"][f])].tolist() for f in range(len(off) - 1)]


def check_frames_equal_plain(den, frames, off, o, dumps, params, which=None):
    """Every frame of the batch (or the frames listed in ``which``) against a
    plain run of that frame."""
    den.set_params(**params)
    for f in (range(len(frames)) if which is None else which):
        fr = frames[f]
        a, b = int(off[f]), int(off[f + 1])
        n = b - a
        g = run_gpu(den, fr)
        tag = f"frame {f} (n={n})"
        assert o["n_kept"][f] == g["n_kept"], tag
        assert np.array_equal(o["keep"][a:b], g["keep"]), tag
        assert np.array_equal(o["score"][a:b].view(np.uint32), g["score"].view(np.uint32)), tag
        assert np.array_equal(o["stage"][a:b], g["stage"]), tag
        assert np.array_equal(o["kept_idx"][a:a + g["n_kept"]], g["kept_idx"]), tag
        if n == 0 or dumps is None:
            continue
        B = {w: v[a:b] for w, v in dumps.items() if w in PER_POINT}
        assert np.array_equal(B["KEYS"].view(np.uint64), g["key"]), tag
        lof = B["LEAF_OF"].view(np.uint32)
        assert np.array_equal(lof - lof.min(), g["leaf_of"]), tag
        lt = dumps["LEAF_TABLE"]
        mine = lt[(lt[:, 0] >= a) & (lt[:, 0] < b)]
        assert len(mine) == g["n_leaves"], tag
        assert np.array_equal(mine[:, 0] - a, g["leaf_begin"]) and np.array_equal(mine[:, 1] - a, g["leaf_end"]), tag
        # the same points in every leaf range (the order inside a leaf is free)
        bo = B["ORDER"].view(np.uint32) - a
        want = np.repeat(np.arange(g["n_leaves"], dtype=np.uint32), (g["leaf_end"] - g["leaf_begin"]).astype(np.int64))
        assert np.array_equal(np.sort(bo), np.arange(n, dtype=np.uint32)), tag
        assert np.array_equal(g["leaf_of"][bo], want) and np.array_equal(g["leaf_of"][g["order"]], want), tag
        assert np.array_equal(mine[:, 2], g["leaf_level"]), tag
        assert np.array_equal(mine[:, 3], g["leaf_h"].view(np.uint32)), tag
        for w, key in (("OCC", "occ"), ("P1", "p1"), ("P2", "p2")):
            assert np.array_equal(B[w].view(g[key].dtype), g[key]), (tag, w)
        nb = B["NBR_IDX"].view(np.uint32).copy()
        nb[nb != 0xFFFFFFFF] -= a
        assert np.array_equal(nb, g["nbr_idx"]), tag
        for w, key in (("NBR_D2", "nbr_d2"), ("R2K", "r2k"), ("RHO", "rho"), ("SCORE64", "score64")):
            x, y = B[w], g[key]
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), (tag, w)


def test_batch_equals_plain_per_frame(bden, den):
    params = dict(k=12, leaf_cap=128)
    frames = frames_mixed()
    xyz, offd, off = to_dev(frames)
    print(f"[batch] frames={[len(f) for f in frames]} params={params}", flush=True)
    bden.set_params(**params)
    res = bden(xyz, offd)
    o = outputs(res, xyz.shape[0], len(frames))
    dumps = batch_dumps(bden, xyz.shape[0], len(frames))
    assert dumps["status"] == 0
    check_frames_equal_plain(den, frames, off, o, dumps, params)


def test_batch_frame_against_oracle(bden, oracle):
    params = dict(k=16, leaf_cap=256)
    frames = [synth.sphere_plane(seed=21, n_sphere=2500, n_plane=800, n_out=600)[0],
              synth.lidar_frame(seed=22, n_az=120)[0]]
    xyz, offd, off = to_dev(frames)
    bden.set_params(**params)
    o = outputs(bden(xyz, offd), xyz.shape[0], 2)
    for f, fr in enumerate(frames):
        ref = oracle.denoise(fr, **params)
        a, b = int(off[f]), int(off[f + 1])
        assert o["n_kept"][f] == ref["n_kept"]
        assert np.array_equal(o["kept_idx"][a:a + ref["n_kept"]], ref["kept_idx"])
        F = ref["score"]
        m = F >= 0
        assert np.allclose(o["score"][a:b][m], F[m], rtol=1e-5, atol=0)


@pytest.mark.parametrize("nframes", [300, 2100])
def test_many_tiny_frames_two_frame_digits(bden, den, nframes):
    # more than 256 frames: the sort takes two frame-id digits; up to 2047
    # frames its frame passes search the offsets in LDS, beyond in memory
    rng = np.random.default_rng(8 if nframes == 300 else nframes)
    sizes = rng.integers(0, 40, nframes)
    frames = [synth.uniform_cube(100 + i, int(s))[0] if s else np.zeros((0, 3), np.float32)
              for i, s in enumerate(sizes)]
    params = dict(k=4, leaf_cap=8, min_vox_count=1)
    xyz, offd, off = to_dev(frames)
    print(f"[batch] {len(frames)} frames, n={xyz.shape[0]}", flush=True)
    bden.set_params(**params)
    o = outputs(bden(xyz, offd), xyz.shape[0], len(frames))
    dumps = batch_dumps(bden, xyz.shape[0], len(frames))
    assert dumps["status"] == 0
    check_frames_equal_plain(den, frames[:40], off, o, dumps, params)
    # the rest: outputs only
    check_frames_equal_plain(den, frames, off, o, None, params)


@pytest.mark.parametrize("nframes", [300, 2100])
def test_many_frames_above_1m_points(bden, den, nframes):
    """More than 256 frames (two frame-id digits) and, with 2100, more than
    2047 (frame offsets searched in memory rather than in LDS), in a batch of
    more than 2^20 points, so the 16-key radix tiles scatter both frame
    digits through LDS and the other large-input kernels run. Sampled frames
    equal their plain runs in every intermediate, the rest in their outputs."""
    beams, az = (16, 232) if nframes == 300 else (8, 88)
    rng = np.random.default_rng(nframes + 1)
    frames = [synth.lidar_frame(seed=5000 + i, n_beams=beams, n_az=int(az + rng.integers(-8, 9)))[0]
              for i in range(nframes)]
    params = dict(k=8, leaf_cap=128)
    xyz, offd, off = to_dev(frames)
    assert xyz.shape[0] > (1 << 20)
    print(f"[batch] {nframes} frames above 1M: n={xyz.shape[0]}", flush=True)
    bden.set_params(**params)
    o = outputs(bden(xyz, offd), xyz.shape[0], len(frames))
    dumps = batch_dumps(bden, xyz.shape[0], len(frames))
    assert dumps["status"] == 0
    sample = sorted(set([0, 1, 255, 256, 257, nframes // 2, nframes - 2, nframes - 1] +
                        list(rng.choice(nframes, 6, replace=False))))
    check_frames_equal_plain(den, frames, off, o, dumps, params, which=sample)
    check_frames_equal_plain(den, frames, off, o, None, params, which=range(0, nframes, 7))


def test_one_frame_batch_equals_plain(bden, den):
    params = dict(k=16, leaf_cap=512)
    fr = synth.sphere_plane(seed=4, n_sphere=2000, n_plane=700, n_out=500)[0]
    xyz, offd, off = to_dev([fr])
    bden.set_params(**params)
    o = outputs(bden(xyz, offd), xyz.shape[0], 1)
    check_frames_equal_plain(den, [fr], off, o, batch_dumps(bden, xyz.shape[0], 1), params)


def test_graph_replays_match_eager(bden, den):
    import torch
    params = dict(k=12, leaf_cap=128)
    frames = frames_mixed()
    xyz, offd, off = to_dev(frames)
    n, nf = xyz.shape[0], len(frames)
    bden.set_params(**params)
    out = bden.alloc(n, nf)
    alt = [synth.uniform_cube(300 + i, len(f))[0] if len(f) else f for i, f in enumerate(frames)]
    xyz_alt = torch.from_numpy(np.concatenate(alt)).cuda()
    keep = xyz.clone()
    for rep, src in enumerate((keep, xyz_alt, keep)):
        xyz.copy_(src)  # same buffer, new contents
        bden.graph(xyz, offd, out)
        got = outputs(out, n, nf)
        eager = outputs(bden(xyz, offd), n, nf)  # eager work between replays
        print(f"[graph] replay {rep}: n_kept={got['n_kept'].tolist()}", flush=True)
        for key in ("keep", "score", "stage", "n_kept"):
            assert np.array_equal(got[key], eager[key]), (rep, key)
        assert kept_lists(got, off) == kept_lists(eager, off), rep
    frames_now = frames
    check_frames_equal_plain(den, frames_now, off, got, None, params)


def test_autotune_choice_is_consistent(bden, den):
    params = dict(k=12, leaf_cap=512)
    frames = [synth.lidar_frame(seed=30 + i, n_az=100)[0] for i in range(3)]
    xyz, offd, off = to_dev(frames)
    bden.set_params(**params)
    table = bden.autotune(xyz, offd, caps=[64, 128, 256], chunks=[4096, 16384], reps=1)
    print(f"[autotune] {table} -> cap {bden.params.leaf_cap} chunk {bden.params.knn_chunk}", flush=True)
    assert len(table) == 6 and all(np.isfinite(v) and v > 0 for v in table.values())
    assert bden.params.leaf_cap in (64, 128, 256) and bden.params.knn_chunk in (4096, 16384)
    assert table[(bden.params.leaf_cap, bden.params.knn_chunk)] == min(table.values())
    o = outputs(bden(xyz, offd), xyz.shape[0], 3)
    check_frames_equal_plain(den, frames, off, o, None,
                             dict(k=12, leaf_cap=bden.params.leaf_cap, knn_chunk=bden.params.knn_chunk))


def test_chunk_length_does_not_change_results(bden):
    params = dict(k=32, leaf_cap=1024)
    frames = [synth.lidar_frame(seed=40, n_az=300)[0]]
    xyz, offd, off = to_dev(frames)
    res = []
    for ch in (512, 4096, 0):
        bden.set_params(knn_chunk=ch, **params)
        res.append(outputs(bden(xyz, offd), xyz.shape[0], 1))
        res[-1]["nbr"] = bden.dump("NBR_IDX", xyz.shape[0]).cpu().numpy()
    for r in res[1:]:
        for key in ("keep", "score", "stage", "n_kept", "nbr"):
            assert np.array_equal(r[key], res[0][key]), key
        assert kept_lists(r, off) == kept_lists(res[0], off)


def test_bad_frame_table_is_repaired_and_flagged(bden):
    import torch
    frames = [synth.uniform_cube(50, 500)[0], synth.uniform_cube(51, 700)[0]]
    xyz, offd, off = to_dev(frames)
    bad = torch.tensor([0, 900, 400], dtype=torch.int64, device="cuda")  # decreasing, wrong end
    bden.set_params(k=8, leaf_cap=64)
    bden(xyz, bad)
    torch.cuda.synchronize()
    st = int(bden.dump("STATUS", xyz.shape[0]).cpu().numpy()[0])
    assert st & 4


def test_empty_batch(bden):
    import torch
    frames = [np.zeros((0, 3), np.float32)] * 3
    xyz, offd, off = to_dev(frames)
    bden.set_params(k=8)
    out = bden.alloc(0, 3)
    out.n_kept.fill_(-1)
    bden(xyz, offd, out)
    torch.cuda.synchronize()
    assert out.n_kept.cpu().tolist() == [0, 0, 0]


@pytest.mark.parametrize("k", [16, 48])
def test_large_batch_paths_equal_plain(bden, den, k):
    # over 1M points: 16-key radix tiles, 16-item scans, the parallel kNN plan,
    # the folded frame boxes, the one-wave selects for leaves <= 256 P1 points
    # and the kNN's position buffers all run here (k = 16: half-wave merges,
    # k = 48: whole-wave merges), and every frame must still equal its plain
    # run (which, under 1M points, takes the other paths)
    params = dict(k=k, leaf_cap=256)
    frames = [synth.lidar_frame(seed=60 + i, n_az=int(n))[0] for i, n in enumerate([1500, 1700, 1300, 1900, 1600,
                                                                                    1800, 1400, 1750, 1650, 1550,
                                                                                    1450, 1850])]
    xyz, offd, off = to_dev(frames)
    assert xyz.shape[0] > (1 << 20)
    print(f"[batch] large: {len(frames)} frames, n={xyz.shape[0]}", flush=True)
    bden.set_params(**params)
    o = outputs(bden(xyz, offd), xyz.shape[0], len(frames))
    dumps = batch_dumps(bden, xyz.shape[0], len(frames))
    assert dumps["status"] == 0
    check_frames_equal_plain(den, frames, off, o, dumps, params)


def test_large_batch_ties_equal_plain(bden, den):
    """Over 1M points with exact duplicates: equal r^2_K, densities and scores
    inside small leaves (the wave radix select and the one-wave voxel filter
    of large batches, against the block paths of the plain runs), clusters of
    more than k identical points (r_K = 0, infinite density) and leaves too
    small to have k candidates (zero density). One frame also holds a tight
    blob whose level-10 cell exceeds the leaf cap (re-sorted on the whole key
    and split below level 10)."""
    params = dict(k=16, leaf_cap=128)
    rng = np.random.default_rng(77)
    frames = []
    for i, n in enumerate([1500, 1700, 1300, 1900, 1600, 1800, 1400, 1750, 1650, 1550, 1450, 1850]):
        fr = synth.lidar_frame(seed=90 + i, n_az=int(n))[0]
        dup = rng.choice(len(fr), len(fr) // 5, replace=False)
        fr[dup] = fr[rng.choice(len(fr), len(dup))]  # a fifth of the points copy others
        fr[:40] = fr[40]  # 41 identical points: r_K = 0 for them
        if i == 3:
            fr[100:2100] = fr[100] + rng.uniform(0, 1e-3, (2000, 3)).astype(np.float32)
        frames.append(fr)
    xyz, offd, off = to_dev(frames)
    assert xyz.shape[0] > (1 << 20)
    print(f"[batch] ties: {len(frames)} frames, n={xyz.shape[0]}", flush=True)
    bden.set_params(**params)
    o = outputs(bden(xyz, offd), xyz.shape[0], len(frames))
    dumps = batch_dumps(bden, xyz.shape[0], len(frames))
    assert dumps["status"] == 0
    rho = dumps["RHO"]
    assert np.isinf(rho).any() and (rho == 0).any()
    assert dumps["LEAF_TABLE"][:, 2].max() > 10  # the blob's leaves lie below level 10
    check_frames_equal_plain(den, frames, off, o, dumps, params)


def test_bench_batch_configuration_sampled_frames_vs_oracle(bden, oracle):
    """The 64-frame LiDAR batch (6.2M points) in the configuration the
    benchmark times after autotuning (leaf cap 256, candidate chunks of
    32768; above 1M points the kNN keeps candidate positions in its buffers):
    three sampled frames against the oracle at the same parameters, down to
    the neighbour lists, and every frame's counts and device status."""
    import torch
    frames, _, params = synth.make("lidar_batch_64")
    params = dict(params, leaf_cap=256, knn_chunk=32768)
    xyz, offd, off = to_dev(frames)
    n, nf = xyz.shape[0], len(frames)
    assert n > (1 << 20)
    bden.set_params(**params)
    res = bden(xyz, offd)
    o = outputs(res, n, nf)
    torch.cuda.synchronize()
    assert int(bden.dump("STATUS", n).cpu().numpy()[0]) == 0
    nbr = bden.dump("NBR_IDX", n).cpu().numpy().view(np.uint32)
    keep = o["keep"]
    for f in range(nf):
        a, b = int(off[f]), int(off[f + 1])
        assert o["n_kept"][f] == int(keep[a:b].sum()), f
    oparams = {k: v for k, v in params.items() if k != "knn_chunk"}
    for f in (0, 31, 63):
        a, b = int(off[f]), int(off[f + 1])
        ref = oracle.denoise(frames[f], **oparams)
        tag = f"frame {f} (n={b - a})"
        p1 = ref["p1"] == 1
        nb = nbr[a:b].copy()
        nb[nb != 0xFFFFFFFF] -= a
        assert np.array_equal(nb[p1], ref["nbr_idx"][p1]), tag
        F = ref["score"]
        m = F >= 0
        assert np.allclose(o["score"][a:b][m], F[m], rtol=1e-5, atol=0), tag
        # keep labels may differ only within the score tolerance of a leaf's cut
        th = leaf_thresholds(ref)
        diff = np.nonzero(keep[a:b] != ref["keep"])[0]
        for i in diff:
            t = ref["leaf_of"][i]
            assert ref["p2"][i] == 1 and abs(F[i] - th[t]) <= 1e-5 * th[t], (tag, i)
        same = keep[a:b] == ref["keep"]
        assert np.array_equal(o["stage"][a:b][same], ref["stage"][same]), tag
