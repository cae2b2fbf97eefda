"""Thin ctypes binding of libgdn.so (include/gdn.h).

The functions named gdn_* mirror the C ABI one to one and only marshal
arguments; every step of the denoiser runs in the library's HIP kernels.
``Denoiser`` adds torch-side allocation of outputs and workspace on the
current stream. Importing this module does not load the library; the first
call does, and raises if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgdn.so")

GDN_OK, GDN_EINVAL, GDN_ENOMEM, GDN_ECAPACITY, GDN_EHIP, GDN_EINTERNAL = range(6)
GDN_DEV_NONFINITE = 1
GDN_DEV_WAIT_LIMIT = 2
GDN_DEV_BAD_FRAMES = 4
GDN_MAX_FRAMES = 4096
GDN_NOALLOC_MAX_BYTES = 192 << 20
GDN_STAGE_VOXEL, GDN_STAGE_DENSITY, GDN_STAGE_SCORE, GDN_STAGES_ALL = 1, 2, 4, 7

DUMP = dict(STATUS=0, COUNTS=1, KEYS=2, ORDER=3, LEAF_OF=4, LEAF_TABLE=5, OCC=6, P1=7,
            NBR_IDX=8, NBR_D2=9, R2K=10, RHO=11, P2=12, LEAF_RHO_MED=13, SCORE64=14,
            LEAF_NCAND=15)


class gdn_params(C.Structure):
    _fields_ = [("k", C.c_int32), ("leaf_cap", C.c_int32),
                ("min_leaf_side", C.c_double), ("beta", C.c_double),
                ("min_vox_count", C.c_int32), ("rho_percentile", C.c_double),
                ("alpha", C.c_double), ("sigma", C.c_double),
                ("eps", C.c_double), ("keep_ratio", C.c_double),
                ("knn_chunk", C.c_int32), ("gamma", C.c_double),
                ("log_threshold", C.c_double), ("stages", C.c_int32)]


class gdn_fit_params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("sigma", C.c_double), ("gamma", C.c_double),
                ("tau", C.c_double), ("temperature", C.c_double)]


class GdnError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"gdn status {status}: {message}")
        self.status = status


_lib = None


def lib():
    """Load libgdn.so; raise if it is missing (there is no fallback path) or
    was built from other sources than the ones beside it."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2512_10386_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.gdn_source_hash.argtypes = []
        L.gdn_source_hash.restype = C.c_char_p
        from . import build as _build
        built, now = L.gdn_source_hash().decode(), _build.source_hash()
        if built != now:
            raise RuntimeError(f"{LIB_PATH} is stale (built from sources {built[:12]}, the tree holds "
                               f"{now[:12]}): rebuild it with `python -m paper_2512_10386_amd.build`")
        vp, i64, sz = C.c_void_p, C.c_int64, C.c_size_t
        L.gdn_default_params.argtypes = [C.POINTER(gdn_params)]
        L.gdn_create.argtypes = [C.POINTER(vp), C.c_int]
        L.gdn_destroy.argtypes = [vp]
        L.gdn_destroy.restype = None
        L.gdn_workspace_size.argtypes = [vp, C.POINTER(gdn_params), i64, C.POINTER(sz)]
        L.gdn_denoise.argtypes = [vp, C.POINTER(gdn_params), vp, i64, vp, sz, vp, vp, vp, vp, vp, vp]
        L.gdn_denoise_noalloc.argtypes = [vp, C.POINTER(gdn_params), vp, i64, vp, vp, vp, vp, vp, vp]
        L.gdn_workspace_size_batch.argtypes = [vp, C.POINTER(gdn_params), i64, i64, C.POINTER(sz)]
        L.gdn_denoise_batch.argtypes = [vp, C.POINTER(gdn_params), vp, i64, vp, i64, vp, sz,
                                        vp, vp, vp, vp, vp, vp]
        L.gdn_graph_create.argtypes = [vp, C.POINTER(gdn_params), vp, i64, vp, i64, vp, sz,
                                       vp, vp, vp, vp, vp, C.POINTER(vp)]
        L.gdn_graph_launch.argtypes = [vp, vp]
        L.gdn_graph_destroy.argtypes = [vp]
        L.gdn_graph_destroy.restype = None
        L.gdn_server_create.argtypes = [vp, C.POINTER(gdn_params), sz, C.c_int, i64, C.c_int, C.POINTER(vp)]
        L.gdn_server_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(sz)]
        L.gdn_server_submit.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, C.POINTER(i64)]
        L.gdn_server_poll.argtypes = [vp, C.POINTER(i64), C.POINTER(C.c_uint32), C.c_int, C.POINTER(C.c_int),
                                      C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.gdn_server_destroy.argtypes = [vp]
        L.gdn_server_destroy.restype = None
        L.gdn_server_last_error.argtypes = [vp]
        L.gdn_server_last_error.restype = C.c_char_p
        L.gdn_autotune.argtypes = [vp, C.POINTER(gdn_params), C.POINTER(C.c_int32), C.c_int,
                                   C.POINTER(C.c_int32), C.c_int, C.c_int, vp, i64, vp, i64, vp, sz,
                                   vp, vp, vp, vp, vp, C.POINTER(C.c_float), vp]
        L.gdn_debug_dump.argtypes = [vp, C.c_int, vp, sz, vp]
        L.gdn_fit_workspace_size.argtypes = [vp, i64, C.POINTER(sz)]
        L.gdn_nearest_workspace_size.argtypes = [vp, i64, C.POINTER(sz)]
        L.gdn_nearest.argtypes = [vp, vp, i64, vp, i64, vp, sz, vp, vp, vp]
        L.gdn_eval_workspace_size.argtypes = [vp, i64, i64, C.POINTER(sz)]
        L.gdn_eval_metrics.argtypes = [vp, vp, i64, vp, i64, vp, sz, vp, vp]
        L.gdn_fit_loss_grad.argtypes = [vp, C.POINTER(gdn_fit_params), vp, vp, i64, vp, sz, vp, vp]
        L.gdn_set_timing.argtypes = [vp, C.c_int]
        L.gdn_timing.argtypes = [vp, i64, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.gdn_status_string.argtypes = [C.c_int]
        L.gdn_status_string.restype = C.c_char_p
        L.gdn_last_error.argtypes = [vp]
        L.gdn_last_error.restype = C.c_char_p
        for f in ("gdn_default_params", "gdn_create", "gdn_workspace_size", "gdn_denoise", "gdn_denoise_noalloc",
                  "gdn_debug_dump", "gdn_set_timing", "gdn_timing", "gdn_workspace_size_batch",
                  "gdn_denoise_batch", "gdn_graph_create", "gdn_graph_launch", "gdn_autotune",
                  "gdn_fit_workspace_size", "gdn_fit_loss_grad", "gdn_nearest_workspace_size",
                  "gdn_nearest", "gdn_eval_workspace_size", "gdn_eval_metrics",
                  "gdn_server_create", "gdn_server_info", "gdn_server_submit", "gdn_server_poll"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(ctx, status):
    if status != GDN_OK:
        msg = lib().gdn_last_error(ctx).decode() if ctx else ""
        if not msg:
            msg = lib().gdn_status_string(status).decode()
        raise GdnError(status, msg)


# ------------------------------------------------------------ C ABI mirror


def gdn_default_params() -> gdn_params:
    p = gdn_params()
    _check(None, lib().gdn_default_params(C.byref(p)))
    return p


def gdn_create(device: int = 0) -> int:
    h = C.c_void_p()
    _check(None, lib().gdn_create(C.byref(h), device))
    return h.value


def gdn_destroy(ctx: int) -> None:
    lib().gdn_destroy(ctx)


def gdn_workspace_size(ctx: int, p: gdn_params, n: int) -> int:
    b = C.c_size_t()
    _check(ctx, lib().gdn_workspace_size(ctx, C.byref(p), n, C.byref(b)))
    return b.value


def gdn_denoise(ctx, p, xyz, n, workspace, workspace_bytes, keep, score, stage,
                kept_idx, n_kept, stream) -> None:
    _check(ctx, lib().gdn_denoise(ctx, C.byref(p), xyz, n, workspace, workspace_bytes,
                                  keep, score, stage, kept_idx, n_kept, stream))


def gdn_denoise_noalloc(ctx, p, xyz, n, keep, score, stage, kept_idx, n_kept, stream) -> None:
    _check(ctx, lib().gdn_denoise_noalloc(ctx, C.byref(p), xyz, n, keep, score, stage, kept_idx, n_kept, stream))


def gdn_workspace_size_batch(ctx: int, p: gdn_params, n: int, nf: int) -> int:
    b = C.c_size_t()
    _check(ctx, lib().gdn_workspace_size_batch(ctx, C.byref(p), n, nf, C.byref(b)))
    return b.value


def gdn_denoise_batch(ctx, p, xyz, n, frame_off, nf, workspace, workspace_bytes, keep, score, stage,
                      kept_idx, n_kept, stream) -> None:
    _check(ctx, lib().gdn_denoise_batch(ctx, C.byref(p), xyz, n, frame_off, nf, workspace, workspace_bytes,
                                        keep, score, stage, kept_idx, n_kept, stream))


def gdn_graph_create(ctx, p, xyz, n, frame_off, nf, workspace, workspace_bytes, keep, score, stage,
                     kept_idx, n_kept) -> int:
    g = C.c_void_p()
    _check(ctx, lib().gdn_graph_create(ctx, C.byref(p), xyz, n, frame_off, nf, workspace, workspace_bytes,
                                       keep, score, stage, kept_idx, n_kept, C.byref(g)))
    return g.value


def gdn_graph_launch(ctx, g, stream) -> None:
    _check(ctx, lib().gdn_graph_launch(g, stream))


def gdn_graph_destroy(g) -> None:
    lib().gdn_graph_destroy(g)


def gdn_autotune(ctx, p, caps, chunks, reps, xyz, n, frame_off, nf, workspace, workspace_bytes, keep, score,
                 stage, kept_idx, n_kept, stream):
    """Tune (leaf_cap, knn_chunk) in place in p; returns the median ms per pair."""
    ca = (C.c_int32 * len(caps))(*caps)
    ch = (C.c_int32 * len(chunks))(*chunks) if chunks else None
    nch = len(chunks) if chunks else 1
    ms = (C.c_float * (len(caps) * nch))()
    _check(ctx, lib().gdn_autotune(ctx, C.byref(p), ca, len(caps), ch, len(chunks) if chunks else 0, reps,
                                   xyz, n, frame_off, nf, workspace, workspace_bytes, keep, score, stage,
                                   kept_idx, n_kept, ms, stream))
    return list(ms)


def _check_srv(srv, status):
    if status != GDN_OK:
        msg = lib().gdn_server_last_error(srv).decode() if srv else ""
        raise GdnError(status, msg or lib().gdn_status_string(status).decode())


def gdn_server_create(ctx, p, hbm_budget, max_slots, slot_points, slot_frames) -> int:
    s = C.c_void_p()
    _check(ctx, lib().gdn_server_create(ctx, C.byref(p), hbm_budget, max_slots, slot_points, slot_frames,
                                        C.byref(s)))
    return s.value


def gdn_server_info(srv):
    ns, b = C.c_int(), C.c_size_t()
    _check_srv(srv, lib().gdn_server_info(srv, C.byref(ns), C.byref(b)))
    return ns.value, b.value


def gdn_server_submit(srv, xyz, n, keep, score, stage, kept_idx, n_kept) -> int:
    t = C.c_int64()
    _check_srv(srv, lib().gdn_server_submit(srv, xyz, n, keep, score, stage, kept_idx, n_kept, C.byref(t)))
    return t.value


def gdn_server_poll(srv, max_done: int = 256):
    """(finished tickets, their batches' device status words, queue length, busy slots)"""
    buf = (C.c_int64 * max_done)()
    sts = (C.c_uint32 * max_done)()
    nd, nw, nb = C.c_int(), C.c_int(), C.c_int()
    _check_srv(srv, lib().gdn_server_poll(srv, buf, sts, max_done, C.byref(nd), C.byref(nw), C.byref(nb)))
    return list(buf[:nd.value]), list(sts[:nd.value]), nw.value, nb.value


def gdn_server_destroy(srv) -> None:
    lib().gdn_server_destroy(srv)


def gdn_fit_workspace_size(ctx, n) -> int:
    b = C.c_size_t()
    _check(ctx, lib().gdn_fit_workspace_size(ctx, n, C.byref(b)))
    return b.value


def gdn_fit_loss_grad(ctx, fp, xyz, label, n, ws, ws_bytes, out, stream) -> None:
    _check(ctx, lib().gdn_fit_loss_grad(ctx, C.byref(fp), xyz, label, n, ws, ws_bytes, out, stream))


def gdn_nearest_workspace_size(ctx, na) -> int:
    b = C.c_size_t()
    _check(ctx, lib().gdn_nearest_workspace_size(ctx, na, C.byref(b)))
    return b.value


def gdn_nearest(ctx, a, na, b, nb, ws, ws_bytes, idx, d2, stream) -> None:
    _check(ctx, lib().gdn_nearest(ctx, a, na, b, nb, ws, ws_bytes, idx, d2, stream))


def gdn_eval_workspace_size(ctx, nc, nd) -> int:
    b = C.c_size_t()
    _check(ctx, lib().gdn_eval_workspace_size(ctx, nc, nd, C.byref(b)))
    return b.value


def gdn_eval_metrics(ctx, clean, nc, den, nd, ws, ws_bytes, out, stream) -> None:
    _check(ctx, lib().gdn_eval_metrics(ctx, clean, nc, den, nd, ws, ws_bytes, out, stream))


def gdn_debug_dump(ctx, what, dst, dst_bytes, stream) -> None:
    _check(ctx, lib().gdn_debug_dump(ctx, what, dst, dst_bytes, stream))


def gdn_set_timing(ctx, enable: bool) -> None:
    _check(ctx, lib().gdn_set_timing(ctx, 1 if enable else 0))


def gdn_timing(ctx, back: int = 0):
    """(whole-call ms, kNN-kernel ms) of a recent timed call."""
    t, k = C.c_float(), C.c_float()
    _check(ctx, lib().gdn_timing(ctx, back, C.byref(t), C.byref(k)))
    return t.value, k.value


def make_params(**kw) -> gdn_params:
    p = gdn_default_params()
    names = {f for f, _ in gdn_params._fields_}
    for key, v in kw.items():
        if key not in names:
            raise TypeError(f"unknown parameter {key!r}")
        setattr(p, key, v)
    return p


# ------------------------------------------------------------ torch wrapper


@dataclass
class Result:
    keep: "object"      # uint8 [n]
    score: "object"     # float32 [n]
    stage: "object"     # uint8 [n]
    kept_idx: "object"  # int32 view of uint32 [n]; first n_kept entries valid
    n_kept: "object"    # int64 [1] device scalar


class Denoiser:
    """One library context plus a reusable workspace on a CUDA (HIP) device."""

    def __init__(self, device: int = 0, **params):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = gdn_create(device)
        self.params = make_params(**params)
        self._ws = None

    def close(self):
        if self.ctx:
            gdn_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **params):
        self.params = make_params(**params)

    def workspace(self, n: int):
        need = gdn_workspace_size(self.ctx, self.params, n)
        if self._ws is None or self._ws.numel() < need:
            self._ws = self.torch.empty(max(need, 256), dtype=self.torch.uint8, device=self.device)
        return self._ws, need

    def __call__(self, xyz, out: Result | None = None) -> Result:
        torch = self.torch
        if xyz.device != self.device or xyz.dtype != torch.float32 or xyz.dim() != 2 or xyz.shape[1] != 3:
            raise ValueError("xyz must be a float32 [n, 3] tensor on the context's device")
        xyz = xyz.contiguous()
        n = xyz.shape[0]
        ws, need = self.workspace(n)
        if out is None:
            out = Result(keep=torch.empty(n, dtype=torch.uint8, device=self.device),
                         score=torch.empty(n, dtype=torch.float32, device=self.device),
                         stage=torch.empty(n, dtype=torch.uint8, device=self.device),
                         kept_idx=torch.empty(max(n, 1), dtype=torch.int32, device=self.device),
                         n_kept=torch.empty(1, dtype=torch.int64, device=self.device))
        stream = torch.cuda.current_stream(self.device).cuda_stream
        gdn_denoise(self.ctx, self.params, xyz.data_ptr(), n, ws.data_ptr(), ws.numel(),
                    out.keep.data_ptr(), out.score.data_ptr(), out.stage.data_ptr(),
                    out.kept_idx.data_ptr(), out.n_kept.data_ptr(), stream)
        return out

    def check_status(self, n: int) -> int:
        """Wait for the last call and raise GdnError if the device flagged a
        condition (GDN_DEV_* bits: non-finite input, an exhausted wait, a bad
        frame table), whose outputs are unspecified. Returns the status word."""
        if n == 0:
            return 0
        st = int(self.dump("STATUS", n).cpu().item())
        if st:
            names = [m for b, m in ((GDN_DEV_NONFINITE, "non-finite coordinates"),
                                    (GDN_DEV_WAIT_LIMIT, "an inter-workgroup wait hit its limit"),
                                    (GDN_DEV_BAD_FRAMES, "bad frame table")) if st & b]
            raise GdnError(GDN_EINTERNAL, f"device status {st:#x}: {', '.join(names)}; outputs unspecified")
        return st

    def dump(self, what: str, n: int):
        """Intermediates of the last frame (original point order), as a tensor."""
        torch = self.torch
        k = self.params.k
        spec = {
            "STATUS": (torch.int32, (1,)), "COUNTS": (torch.int64, (4,)),
            "KEYS": (torch.int64, (n,)), "ORDER": (torch.int32, (n,)),
            "LEAF_OF": (torch.int32, (n,)), "LEAF_TABLE": (torch.int32, (n, 4)),
            "OCC": (torch.int32, (n,)), "P1": (torch.uint8, (n,)),
            "NBR_IDX": (torch.int32, (n, k)), "NBR_D2": (torch.float32, (n, k)),
            "R2K": (torch.float32, (n,)), "RHO": (torch.float64, (n,)),
            "P2": (torch.uint8, (n,)), "LEAF_RHO_MED": (torch.float64, (n,)),
            "SCORE64": (torch.float64, (n,)), "LEAF_NCAND": (torch.int32, (n,)),
        }
        dt, shape = spec[what]
        t = torch.empty(shape, dtype=dt, device=self.device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        gdn_debug_dump(self.ctx, DUMP[what], t.data_ptr(), t.numel() * t.element_size(), stream)
        return t


class BatchDenoiser(Denoiser):
    """Batches of frames through gdn_denoise_batch, optionally replayed from a
    captured HIP graph (same batch shape, new contents)."""

    def __init__(self, device: int = 0, **params):
        super().__init__(device, **params)
        self._graph = None
        self._graph_key = None

    def close(self):
        self.drop_graph()
        super().close()

    def drop_graph(self):
        if self._graph:
            gdn_graph_destroy(self._graph)
        self._graph = None
        self._graph_key = None

    def workspace_batch(self, n: int, nf: int):
        need = gdn_workspace_size_batch(self.ctx, self.params, n, nf)
        if self._ws is None or self._ws.numel() < need:
            self.drop_graph()  # a graph holds the old workspace's address
            self._ws = self.torch.empty(max(need, 256), dtype=self.torch.uint8, device=self.device)
        return self._ws, need

    def alloc(self, n: int, nf: int) -> Result:
        torch = self.torch
        return Result(keep=torch.empty(max(n, 1), dtype=torch.uint8, device=self.device),
                      score=torch.empty(max(n, 1), dtype=torch.float32, device=self.device),
                      stage=torch.empty(max(n, 1), dtype=torch.uint8, device=self.device),
                      kept_idx=torch.empty(max(n, 1), dtype=torch.int32, device=self.device),
                      n_kept=torch.empty(max(nf, 1), dtype=torch.int64, device=self.device))

    def _check_inputs(self, xyz, frame_off):
        torch = self.torch
        if xyz.device != self.device or xyz.dtype != torch.float32 or xyz.dim() != 2 or xyz.shape[1] != 3:
            raise ValueError("xyz must be a float32 [n, 3] tensor on the context's device")
        if frame_off.device != self.device or frame_off.dtype != torch.int64 or frame_off.dim() != 1:
            raise ValueError("frame_off must be an int64 [nf + 1] tensor on the context's device")
        if not xyz.is_contiguous() or not frame_off.is_contiguous():
            raise ValueError("xyz and frame_off must be contiguous")

    def __call__(self, xyz, frame_off, out: Result | None = None) -> Result:
        self._check_inputs(xyz, frame_off)
        n, nf = xyz.shape[0], frame_off.shape[0] - 1
        ws, _ = self.workspace_batch(n, nf)
        if out is None:
            out = self.alloc(n, nf)
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        gdn_denoise_batch(self.ctx, self.params, xyz.data_ptr(), n, frame_off.data_ptr(), nf, ws.data_ptr(),
                          ws.numel(), out.keep.data_ptr(), out.score.data_ptr(), out.stage.data_ptr(),
                          out.kept_idx.data_ptr(), out.n_kept.data_ptr(), stream)
        return out

    def graph(self, xyz, frame_off, out: Result):
        """Capture (once per batch shape and buffers) and launch the batch."""
        self._check_inputs(xyz, frame_off)
        n, nf = xyz.shape[0], frame_off.shape[0] - 1
        ws, _ = self.workspace_batch(n, nf)
        key = (n, nf, xyz.data_ptr(), frame_off.data_ptr(), ws.data_ptr(), out.keep.data_ptr(),
               out.score.data_ptr(), out.stage.data_ptr(), out.kept_idx.data_ptr(), out.n_kept.data_ptr(),
               bytes(self.params))
        if self._graph_key != key:
            self.drop_graph()
            self._graph = gdn_graph_create(self.ctx, self.params, xyz.data_ptr(), n, frame_off.data_ptr(), nf,
                                           ws.data_ptr(), ws.numel(), out.keep.data_ptr(), out.score.data_ptr(),
                                           out.stage.data_ptr(), out.kept_idx.data_ptr(), out.n_kept.data_ptr())
            self._graph_key = key
        gdn_graph_launch(self.ctx, self._graph, self.torch.cuda.current_stream(self.device).cuda_stream)
        return out

    def autotune(self, xyz, frame_off, caps, chunks=None, reps=3):
        """Pick (leaf_cap, knn_chunk) for this batch; returns {(cap, chunk): ms}."""
        self._check_inputs(xyz, frame_off)
        n, nf = xyz.shape[0], frame_off.shape[0] - 1
        ws, _ = self.workspace_batch(n, nf)
        out = self.alloc(n, nf)
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        ms = gdn_autotune(self.ctx, self.params, list(caps), list(chunks or []), reps, xyz.data_ptr(), n,
                          frame_off.data_ptr(), nf, ws.data_ptr(), ws.numel(), out.keep.data_ptr(),
                          out.score.data_ptr(), out.stage.data_ptr(), out.kept_idx.data_ptr(),
                          out.n_kept.data_ptr(), stream)
        self.drop_graph()
        chs = list(chunks) if chunks else [0]
        return {(c, h): ms[a * len(chs) + b] for a, c in enumerate(caps) for b, h in enumerate(chs)}
