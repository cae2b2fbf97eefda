"""Evaluation of denoised clouds and the module ablation (Sec. 4.1, 4.3.2).

``Evaluator`` runs the library's exact nearest-neighbour and metric kernels
(gdn_nearest, gdn_eval_metrics): PSNR (Eq. 29) and the Chamfer distance
(Eq. 30) of a denoised cloud against the clean one. ``ablation`` runs one
labelled frame through the switch combinations of Tables 8 and 9 and reports
F1 (Eq. 26-28), PSNR, CD and the GPU time per frame for each.
"""
from __future__ import annotations

import statistics

import numpy as np

from . import binding as B
from .fit import f1_scores

# (name, stages, octree) rows: Table 9's module combinations with the octree,
# and Table 8's full method without it (one leaf holding the whole frame).
# The paper's "Baseline" row is its Sec. 2.2 method, which is not built here;
# the row with every module off is the octree + kNN skeleton keeping every
# point with k neighbours.
ABLATION_ROWS = [
    ("none", 0, True), ("A1", 1, True), ("A2", 2, True), ("A3", 4, True),
    ("A1+A2", 3, True), ("A1+A3", 5, True), ("A2+A3", 6, True), ("A1+A2+A3", 7, True),
    ("A1+A2+A3 no octree", 7, False),
]


class Evaluator:
    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = B.gdn_create(device)

    def close(self):
        if self.ctx:
            B.gdn_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def nearest(self, a, b):
        """Nearest point of b for every point of a: (idx int32 view of uint32, fp32 d2)."""
        t = self.torch
        na, nb = a.shape[0], b.shape[0]
        need = B.gdn_nearest_workspace_size(self.ctx, na)
        ws = t.empty(need, dtype=t.uint8, device=self.device)
        idx = t.empty(na, dtype=t.int32, device=self.device)
        d2 = t.empty(na, dtype=t.float32, device=self.device)
        B.gdn_nearest(self.ctx, a.data_ptr(), na, b.data_ptr(), nb, ws.data_ptr(), need, idx.data_ptr(),
                      d2.data_ptr(), self._stream())
        return idx, d2

    def metrics(self, clean, den):
        """Device float64 [4]: MSE, mean denoised->clean, CD (Eq. 30), PSNR dB (Eq. 29)."""
        t = self.torch
        nc, nd = clean.shape[0], den.shape[0]
        need = B.gdn_eval_workspace_size(self.ctx, nc, nd)
        ws = t.empty(need, dtype=t.uint8, device=self.device)
        out = t.empty(4, dtype=t.float64, device=self.device)
        B.gdn_eval_metrics(self.ctx, clean.data_ptr(), nc, den.data_ptr(), nd, ws.data_ptr(), need,
                           out.data_ptr(), self._stream())
        return out


def ablation(xyz: np.ndarray, label: np.ndarray, params: dict, reps: int = 10, rows=ABLATION_ROWS,
             device: int = 0):
    """Rows of (name, stages, leaf_cap, precision, recall, F1, PSNR dB, CD,
    ms per frame) for one labelled frame; the clean cloud is the label-0 points."""
    import torch
    dev = torch.device("cuda", device)
    x = torch.from_numpy(np.ascontiguousarray(xyz, np.float32)).to(dev)
    clean = torch.from_numpy(np.ascontiguousarray(xyz[label == 0], np.float32)).to(dev)
    ev = Evaluator(device)
    out = []
    try:
        for name, stages, octree in rows:
            prm = dict(params, stages=stages)
            if not octree:
                prm["leaf_cap"] = max(int(xyz.shape[0]), 1)
            den = B.Denoiser(device, **prm)
            try:
                res = den(x)
                ms = []
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                for _ in range(reps):
                    e0.record()
                    den(x, res)
                    e1.record()
                    e1.synchronize()
                    ms.append(e0.elapsed_time(e1))
                keep = res.keep.cpu().numpy()
            finally:
                den.close()
            p, r, f = f1_scores(keep, label)
            kept = x[torch.from_numpy(keep.astype(bool)).to(dev)].contiguous()
            if kept.shape[0] > 0:
                m = ev.metrics(clean, kept).cpu().numpy()
                psnr, cd = float(m[3]), float(m[2])
            else:
                psnr, cd = float("nan"), float("nan")
            out.append(dict(name=name, stages=stages, leaf_cap=prm["leaf_cap"], precision=p, recall=r, f1=f,
                            psnr_db=psnr, cd=cd, ms=statistics.median(ms)))
    finally:
        ev.close()
    return out
