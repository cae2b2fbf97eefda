"""Score fit: gradient-based fitting of the weight parameters of Eq. 17-21.

``ScoreFit`` runs the pipeline once on labelled frames (a batch is fine) and
then evaluates, on the GPU, the loss of a relaxed threshold on ln F_i and its
gradient over (alpha, sigma, gamma, tau) with the library's fit kernel
(gdn_fit_loss_grad); the neighbour sets, densities, medians and P2 stay those
of that pass. ``ScoreLoss`` wraps it as a torch autograd function, so any
torch optimiser can drive the parameters. ``f1_scores`` gives the precision,
recall and F1 of noise removal (Eq. 26-28).
"""
from __future__ import annotations

import functools

import numpy as np

from . import binding as B


class ScoreFit:
    """Labelled frames, denoised once; loss/gradient evaluations on demand.

    xyz: float32 [n, 3] device tensor (frames back to back), label: uint8 [n]
    (1 = noise), frame_off: int64 [nf + 1] device tensor or None (one frame).
    """

    def __init__(self, xyz, label, frame_off=None, temperature: float = 1.0, device: int = 0, **params):
        import torch
        self.torch = torch
        self.n = xyz.shape[0]
        self.xyz = xyz.contiguous()
        self.label = label.contiguous()
        self.temperature = float(temperature)
        if frame_off is None:
            self.den = B.Denoiser(device, **params)
            self.res = self.den(self.xyz)
        else:
            self.den = B.BatchDenoiser(device, **params)
            self.res = self.den(self.xyz, frame_off)
        need = B.gdn_fit_workspace_size(self.den.ctx, self.n)
        self.ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.xyz.device)
        self.out = torch.empty(6, dtype=torch.float64, device=self.xyz.device)

    def close(self):
        self.den.close()

    def loss_grad(self, alpha: float, sigma: float, gamma: float, tau: float):
        """Device float64 [6]: loss, dL/dalpha, dL/dsigma, dL/dgamma, dL/dtau, terms."""
        fp = B.gdn_fit_params(alpha=alpha, sigma=sigma, gamma=gamma, tau=tau, temperature=self.temperature)
        stream = self.torch.cuda.current_stream(self.xyz.device).cuda_stream
        B.gdn_fit_loss_grad(self.den.ctx, fp, self.xyz.data_ptr(), self.label.data_ptr(), self.n,
                            self.ws.data_ptr(), self.ws.numel(), self.out.data_ptr(), stream)
        return self.out


@functools.lru_cache(maxsize=None)
def _loss_fn():
    import torch

    class ScoreLoss(torch.autograd.Function):
        """loss = ScoreLoss.apply(theta, fit), theta = (alpha, sigma, gamma, tau)
        as a float64 tensor; the backward returns the kernel's gradient."""

        @staticmethod
        def forward(ctx, theta, fit):
            a, s, g, t = (float(v) for v in theta.detach().cpu().tolist())
            out = fit.loss_grad(a, s, g, t).to(theta.device, copy=True)
            ctx.save_for_backward(out[1:5].to(theta.dtype))
            return out[0].to(theta.dtype)

        @staticmethod
        def backward(ctx, grad):
            (g,) = ctx.saved_tensors
            return grad * g, None

    return ScoreLoss


def score_loss(theta, fit: ScoreFit):
    """Differentiable loss of ``fit`` at theta = (alpha, sigma, gamma, tau)."""
    return _loss_fn().apply(theta, fit)


def fit_params(fit: ScoreFit, theta0, steps: int = 100, lr: float = 0.05, min_sigma: float = 1e-3):
    """Adam over theta = (alpha, sigma, gamma, tau); alpha and gamma are kept
    >= 0 and sigma >= min_sigma after every step. Returns (theta, losses)."""
    import torch
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([theta], lr=lr)
    losses = []
    for _ in range(steps):
        opt.zero_grad()
        loss = score_loss(theta, fit)
        loss.backward()
        opt.step()
        with torch.no_grad():
            theta[0].clamp_(min=0.0)
            theta[1].clamp_(min=min_sigma)
            theta[2].clamp_(min=0.0)
        losses.append(float(loss.detach()))
    return [float(v) for v in theta.detach()], losses


def f1_scores(keep: np.ndarray, label: np.ndarray):
    """Precision, recall and F1 of noise removal (Eq. 26-28): removed points
    are the detections, label 1 marks true noise."""
    removed = np.asarray(keep) == 0
    noise = np.asarray(label) == 1
    nq = int(np.sum(removed & noise))
    ns = int(np.sum(removed))
    ny = int(np.sum(noise))
    p = nq / ns if ns else 0.0
    r = nq / ny if ny else 0.0
    f = 2 * p * r / (p + r) if p + r > 0 else 0.0
    return p, r, f
