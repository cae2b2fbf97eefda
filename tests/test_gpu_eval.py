"""Module switches (Table 9) and evaluation kernels (Eq. 29, 30) through the
C ABI, against the oracle.

Switches: every combination runs the whole pipeline and is compared with the
oracle at the same switches by the usual parity bar (bit-exact discrete
results, scores to 1e-5). Nearest neighbours: indices and fp32 distances
bit-exact (same fp32 expression, ties to the smaller index). Metrics: FP64
sums in a different order, relative 1e-12.
"""
import math

import numpy as np
import pytest

from paper_2512_10386_amd import synth
from tests.parity import compare, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ev():
    from paper_2512_10386_amd.evaluate import Evaluator
    e = Evaluator(0)
    yield e
    e.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("stages", list(range(8)))
def test_stage_switches_vs_oracle(oracle, stages):
    from paper_2512_10386_amd.binding import Denoiser
    xyz, _, prm = synth.make("sphere_plane_20k")
    prm = dict(prm, stages=stages)
    ref = oracle.denoise(xyz, **prm)
    den = Denoiser(0, **prm)
    try:
        g = run_gpu(den, xyz)
    finally:
        den.close()
    compare(g, ref)
    if not stages & 4:
        assert np.all(g["score"] == -1.0)
        assert np.array_equal(g["keep"], ref["p2"])


@pytest.mark.parametrize("na,nb", [(1, 1), (1, 5000), (3001, 1), (3001, 4999), (20000, 70000)])
def test_nearest_vs_oracle(ev, oracle, na, nb):
    rng = np.random.default_rng(na * 7 + nb)
    a = rng.uniform(-1, 1, (na, 3)).astype(np.float32)
    b = rng.uniform(-1, 1, (nb, 3)).astype(np.float32)
    # ties: some queries sit on reference points, some references are duplicated
    if nb > 10 and na > 10:
        a[:10] = b[:10]
        b[nb // 2:nb // 2 + 5] = b[:5]
    idx, d2 = ev.nearest(dev(a), dev(b))
    ri, rd = oracle.nearest(a, b)
    assert np.array_equal(idx.cpu().numpy().view(np.uint32), ri)
    assert np.array_equal(d2.cpu().numpy().view(np.uint32), rd.view(np.uint32))


def test_nearest_lattice_ties(ev, oracle):
    """Queries at the centres of lattice cells: 8 equidistant references, the
    smallest index wins on both sides."""
    g = np.arange(6, dtype=np.float32)
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    q = (lat[:125] % 5 + 0.5).astype(np.float32)
    idx, d2 = ev.nearest(dev(q), dev(lat))
    ri, rd = oracle.nearest(q, lat)
    assert np.array_equal(idx.cpu().numpy().view(np.uint32), ri)
    assert np.all(d2.cpu().numpy() == 0.75)


def test_nearest_full_lidar_sampled(ev, oracle):
    """A full 120k LiDAR frame against its 90%-subsample, checked on 2000
    sampled queries by the oracle."""
    xyz, _, _ = synth.make("lidar_120k")
    rng = np.random.default_rng(9)
    b = xyz[rng.random(len(xyz)) < 0.9]
    idx, d2 = ev.nearest(dev(xyz), dev(b))
    s = rng.choice(len(xyz), 2000, replace=False)
    ri, rd = oracle.nearest(xyz[s], b)
    assert np.array_equal(idx.cpu().numpy().view(np.uint32)[s], ri)
    assert np.array_equal(d2.cpu().numpy()[s].view(np.uint32), rd.view(np.uint32))


def test_metrics_vs_oracle(ev, oracle):
    xyz, label = synth.sphere_plane(seed=5, n_sphere=6000, n_plane=2000, n_out=1500)
    clean = xyz[label == 0]
    rng = np.random.default_rng(2)
    den = xyz[rng.random(len(xyz)) < 0.8]
    got = ev.metrics(dev(clean), dev(den)).cpu().numpy()
    exp = oracle.eval_metrics(clean, den)
    assert np.allclose(got, exp, rtol=1e-12, atol=0)


def test_metrics_shifted_lattice(ev):
    m = 9
    g = np.arange(m, dtype=np.float32)
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    delta = np.array([0.125, -0.0625, 0.25], np.float32)
    out = ev.metrics(dev(x), dev(x + delta)).cpu().numpy()
    d2 = float(np.sum(delta.astype(np.float64) ** 2))
    assert out[0] == pytest.approx(d2, rel=1e-14) and out[2] == pytest.approx(2 * d2, rel=1e-14)
    assert out[3] == pytest.approx(10 * math.log10(3 * (m - 1) ** 2 / d2), rel=1e-13)
    same = ev.metrics(dev(x), dev(x)).cpu().numpy()
    assert same[2] == 0.0 and math.isinf(same[3])


def test_eval_errors(ev):
    from paper_2512_10386_amd import binding as B
    with pytest.raises(B.GdnError) as e:
        B.gdn_eval_workspace_size(ev.ctx, 0, 10)
    assert e.value.status == B.GDN_EINVAL
    with pytest.raises(B.GdnError) as e:
        B.gdn_nearest_workspace_size(ev.ctx, 1 << 30)
    assert e.value.status == B.GDN_ECAPACITY


def test_ablation_rows_run():
    from paper_2512_10386_amd.evaluate import ablation
    xyz, label = synth.sphere_plane(seed=6, n_sphere=3000, n_plane=1000, n_out=800)
    rows = ablation(xyz, label, dict(k=16, leaf_cap=512), reps=2)
    assert [r["name"] for r in rows][-2:] == ["A1+A2+A3", "A1+A2+A3 no octree"]
    for r in rows:
        assert 0.0 <= r["f1"] <= 1.0 and r["ms"] > 0
