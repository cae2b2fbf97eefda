"""Pins of the oracle's score-fit additions: the kernel exponent gamma (Eq. 20
is gamma = 2), the threshold keep mode on ln F, and the fit loss with its
gradient over alpha, sigma, gamma and tau (Eq. 17-21 with fixed neighbour
sets, densities, medians and P2).

The checks are closed forms of symmetric configurations, the hand-worked
4-point example, the pinned Eq. 21 score of the plain pipeline, and central
finite differences of the loss.
"""
import math

import numpy as np
import pytest

from paper_2512_10386_amd import synth

TETRA = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], np.float32)  # edge^2 = 8
FOUR = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 3]], np.float32)
# scores of the 4-point example (K=2, alpha=1, sigma=1, eps=0), derived by hand from Eq. 13, 16, 21
FOUR_F = [1.22252420137, 1.19098412647, 0.319415369094, 0.085865175989]


def sig(z):
    return 1.0 / (1.0 + math.exp(-z))


@pytest.mark.parametrize("gamma,kern", [(2.0, 1 / 8), (4.0, 1 / 64), (0.0, 1.0), (3.0, 8.0 ** -1.5)])
def test_kernel_exponent_tetrahedron(oracle, gamma, kern):
    """Every neighbour at d^2 = 8 = r_K^2: F = 3 e^{-1/2} 8^{-gamma/2}."""
    r = oracle.denoise(TETRA, k=3, leaf_cap=10, min_vox_count=1, rho_percentile=0.0,
                       alpha=1.0, sigma=1.0, eps=0.0, keep_ratio=1.0, gamma=gamma)
    assert np.allclose(r["score"], 3.0 * math.exp(-0.5) * kern, rtol=1e-14)


@pytest.mark.parametrize("thr,kept", [(math.log(0.5), [0, 1]), (math.log(0.2), [0, 1, 2]),
                                      (math.log(2.0), []), (math.log(0.05), [0, 1, 2, 3])])
def test_threshold_mode_four_point(oracle, thr, kept):
    r = oracle.denoise(FOUR, k=2, leaf_cap=4, min_vox_count=1, rho_percentile=0.0,
                       alpha=1.0, sigma=1.0, eps=0.0, keep_ratio=0.5, log_threshold=thr)
    assert np.allclose(r["score"], FOUR_F, rtol=1e-10)
    assert list(r["kept_idx"]) == kept
    assert list(r["stage"]) == [3 if i in kept else 2 for i in range(4)]


def test_threshold_mode_rejects_infinite_threshold(oracle):
    with pytest.raises(ValueError):
        oracle.denoise(FOUR, k=2, log_threshold=math.inf)


def test_fit_tetrahedron_closed_form(oracle):
    """All densities equal (w_den = 1), d = r_K for every neighbour:
    F = 3 exp(-1/(2 sigma^2)) 8^{-gamma/2}, so d lnF/d alpha = 0,
    d lnF/d sigma = 1/sigma^3, d lnF/d gamma = -ln(8)/2. Two clean and two
    noise points: dL/dtheta = mean(p - y)/T * d lnF/dtheta, dL/dtau = -mean(p - y)/T."""
    alpha, sigma, gamma, tau, T = 1.3, 0.7, 2.5, -1.0, 0.8
    label = np.array([0, 0, 1, 1], np.uint8)
    r = oracle.denoise(TETRA, k=3, leaf_cap=10, min_vox_count=1, rho_percentile=0.0,
                       alpha=alpha, sigma=sigma, eps=0.0, keep_ratio=1.0, gamma=gamma)
    out = oracle.fit_loss_grad(TETRA, r, label, alpha, sigma, gamma, tau, T)
    lnF = math.log(3.0) - 1.0 / (2 * sigma * sigma) - gamma / 2 * math.log(8.0)
    assert np.allclose(np.log(r["score"]), lnF, rtol=1e-14)
    z = (lnF - tau) / T
    p = sig(z)
    y = np.array([1.0, 1.0, 0.0, 0.0])
    L = float(np.mean(np.log1p(math.exp(z)) - y * z))
    gbar = float(np.mean(p - y)) / T
    assert out[5] == 4
    assert out[0] == pytest.approx(L, rel=1e-13)
    assert out[1] == pytest.approx(0.0, abs=1e-15)
    assert out[2] == pytest.approx(gbar / sigma ** 3, rel=1e-12)
    assert out[3] == pytest.approx(gbar * (-0.5 * math.log(8.0)), rel=1e-12)
    assert out[4] == pytest.approx(-gbar, rel=1e-12)


def test_fit_loss_is_bce_of_the_pipeline_score(oracle):
    """At the pipeline's own alpha, sigma and gamma = 2 the fit's F_i are the
    (pinned) Eq. 21 scores, so the loss is the mean BCE of sigmoid((ln F - tau)/T)."""
    xyz, label = synth.sphere_plane(seed=7, n_sphere=1500, n_plane=500, n_out=400)
    prm = dict(k=10, leaf_cap=256, alpha=1.0, sigma=1.0)
    r = oracle.denoise(xyz, **prm)
    F = r["score"][r["p2"] == 1]
    y = 1.0 - label[r["p2"] == 1].astype(np.float64)
    tau = float(np.median(np.log(F)))
    T = 0.5
    z = (np.log(F) - tau) / T
    L = float(np.mean(np.logaddexp(0.0, z) - y * z))
    out = oracle.fit_loss_grad(xyz, r, label, 1.0, 1.0, 2.0, tau, T)
    assert out[5] == len(F)
    assert out[0] == pytest.approx(L, rel=1e-12)


@pytest.mark.parametrize("case", ["four_point", "sphere_plane"])
def test_fit_gradient_matches_central_differences(oracle, case):
    if case == "four_point":
        xyz = FOUR
        label = np.array([0, 0, 1, 1], np.uint8)
        r = oracle.denoise(xyz, k=2, leaf_cap=4, min_vox_count=1, rho_percentile=0.0, eps=0.0, keep_ratio=0.5)
        theta = dict(alpha=0.9, sigma=1.4, gamma=2.3, tau=-0.5, T=0.7)
    else:
        xyz, label = synth.sphere_plane(seed=8, n_sphere=1200, n_plane=400, n_out=300)
        r = oracle.denoise(xyz, k=12, leaf_cap=200)
        F = r["score"][r["p2"] == 1]
        theta = dict(alpha=1.2, sigma=0.8, gamma=1.7, tau=float(np.median(np.log(F))) + 0.3, T=0.6)

    def loss(**kw):
        a = dict(theta, **kw)
        return oracle.fit_loss_grad(xyz, r, label, a["alpha"], a["sigma"], a["gamma"], a["tau"], a["T"])

    g = loss()
    assert g[5] > 0
    for slot, name in enumerate(["alpha", "sigma", "gamma", "tau"], start=1):
        h = 1e-5 * max(1.0, abs(theta[name]))
        fd = (loss(**{name: theta[name] + h})[0] - loss(**{name: theta[name] - h})[0]) / (2 * h)
        assert g[slot] == pytest.approx(fd, rel=2e-6, abs=1e-9), name


def test_fit_rejects_bad_temperature(oracle):
    r = oracle.denoise(FOUR, k=2, leaf_cap=4, min_vox_count=1, rho_percentile=0.0)
    with pytest.raises(ValueError):
        oracle.fit_loss_grad(FOUR, r, np.zeros(4, np.uint8), 1.0, 1.0, 2.0, 0.0, 0.0)
