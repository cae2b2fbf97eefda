"""Pins of the oracle's ablation flags (the module switches of Table 9) and
its evaluation metrics (PSNR, Eq. 29; Chamfer distance, Eq. 30).

The nearest-neighbour step is checked against scipy's k-d tree and hand
cases; the metrics against closed forms of shifted and thinned lattices; the
flags against the parameter settings they must coincide with (occupancy is
always >= 1, the percentile rank with q = 0 keeps every sufficient point,
lambda = 1 keeps all of P2) and against their direct definitions.
"""
import math

import numpy as np
import pytest

from paper_2512_10386_amd import synth


def lattice(m, spacing=1.0):
    g = np.arange(m, dtype=np.float64) * spacing
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)


# ------------------------------------------------------------- nearest


def test_nearest_hand_case_and_ties(oracle):
    a = np.array([[0, 0, 0], [0.9, 0, 0]], np.float32)
    b = np.array([[1, 0, 0], [-1, 0, 0], [0, 2, 0]], np.float32)
    idx, d2 = oracle.nearest(a, b)
    assert list(idx) == [0, 0]  # (0,0,0): tie between b0 and b1 -> smaller index
    dx = np.float32(1.0) - np.float32(0.9)
    assert d2[0] == 1.0 and d2[1] == dx * dx


def test_nearest_matches_kdtree(oracle):
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(3)
    a = rng.uniform(-1, 1, (3000, 3)).astype(np.float32)
    b = rng.uniform(-1, 1, (2000, 3)).astype(np.float32)
    idx, d2 = oracle.nearest(a, b)
    dist, ref = cKDTree(b.astype(np.float64)).query(a.astype(np.float64), k=2)
    # where the two nearest are well separated the answer is unique
    clear = dist[:, 1] - dist[:, 0] > 1e-4
    assert clear.mean() > 0.9
    assert np.array_equal(idx[clear], ref[clear, 0])
    assert np.allclose(d2, dist[:, 0] ** 2, rtol=1e-5, atol=1e-9)


def test_nearest_rejects_empty_reference(oracle):
    with pytest.raises(ValueError):
        oracle.nearest(np.zeros((3, 3), np.float32), np.zeros((0, 3), np.float32))


# ------------------------------------------------------------- metrics


def test_metrics_identical_clouds(oracle):
    x = lattice(6)
    out = oracle.eval_metrics(x, x)
    assert out[0] == 0.0 and out[1] == 0.0 and out[2] == 0.0 and math.isinf(out[3])


def test_metrics_shifted_lattice_closed_form(oracle):
    """A unit lattice shifted by a dyadic delta (|delta| < 1/2): every point's
    nearest is its own shifted copy, so MSE = |delta|^2, CD = 2 |delta|^2 and
    PSNR = 10 log10(M^2 / |delta|^2), M = sqrt(3) (m - 1)."""
    m = 7
    x = lattice(m)
    delta = np.array([0.125, 0.0625, -0.25], np.float32)
    y = (x + delta).astype(np.float32)
    d2 = float(np.sum(delta.astype(np.float64) ** 2))
    out = oracle.eval_metrics(x, y)
    assert out[0] == pytest.approx(d2, rel=1e-15)
    assert out[1] == pytest.approx(d2, rel=1e-15)
    assert out[2] == pytest.approx(2 * d2, rel=1e-15)
    assert out[3] == pytest.approx(10 * math.log10(3 * (m - 1) ** 2 / d2), rel=1e-14)


def test_metrics_thinned_line_closed_form(oracle):
    """Points 0..n-1 on a line, the odd ones removed: kept points are exact
    matches (den->clean 0); each removed point is 1 from a kept one, so
    MSE = #odd / n."""
    n = 101
    x = np.zeros((n, 3), np.float32)
    x[:, 0] = np.arange(n)
    y = x[::2]
    out = oracle.eval_metrics(x, y)
    assert out[0] == pytest.approx((n // 2) / n, rel=1e-15)
    assert out[1] == 0.0
    assert out[3] == pytest.approx(10 * math.log10((n - 1) ** 2 / ((n // 2) / n)), rel=1e-14)


# ------------------------------------------------------------- ablation flags


@pytest.fixture(scope="module")
def cloud():
    xyz, lab = synth.sphere_plane(seed=12, n_sphere=3000, n_plane=1000, n_out=800)
    return xyz, lab


def test_a1_off_is_voxel_threshold_one(oracle, cloud):
    xyz, _ = cloud
    r = oracle.denoise(xyz, k=10, leaf_cap=256, stages=6)
    s = oracle.denoise(xyz, k=10, leaf_cap=256, min_vox_count=1)
    assert np.all(r["p1"] == 1)
    for f in ("p1", "p2", "keep", "stage"):
        assert np.array_equal(r[f], s[f]), f
    assert np.array_equal(r["score"], s["score"])


def test_a2_off_keeps_every_sufficient_point(oracle, cloud):
    xyz, _ = cloud
    r = oracle.denoise(xyz, k=10, leaf_cap=256, stages=5)
    suff = (r["p1"] == 1) & np.isfinite(np.where(r["p1"] == 1, r["r2k"], np.inf))
    assert np.array_equal(r["p2"] == 1, suff)
    s = oracle.denoise(xyz, k=10, leaf_cap=256, rho_percentile=0.0)
    for f in ("p2", "keep", "stage"):
        assert np.array_equal(r[f], s[f]), f


def test_a3_off_keeps_p2_unscored(oracle, cloud):
    xyz, _ = cloud
    r = oracle.denoise(xyz, k=10, leaf_cap=256, stages=3)
    assert np.array_equal(r["keep"], r["p2"])
    assert np.all(r["score"] == -1.0)
    assert np.array_equal(r["stage"] == 3, r["p2"] == 1)
    s = oracle.denoise(xyz, k=10, leaf_cap=256, keep_ratio=1.0)
    assert np.array_equal(r["keep"], s["keep"])


def test_all_modules_off(oracle, cloud):
    xyz, _ = cloud
    r = oracle.denoise(xyz, k=10, leaf_cap=256, stages=0)
    assert np.all(r["p1"] == 1)
    assert np.array_equal(r["keep"] == 1, np.isfinite(r["r2k"]))


def test_stage_flags_are_validated(oracle, cloud):
    xyz, _ = cloud
    with pytest.raises(ValueError):
        oracle.denoise(xyz[:10], stages=8)
