"""ctypes wrapper of the CPU oracle (gdn_oracle.c).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU-baseline
leg of the benchmark. The product path never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "gdn_oracle.c")]

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
          "-Wno-unused-parameter"]


def build(quiet: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, no FMA contraction)."""
    cmd = ["gcc", *CFLAGS, *SOURCES, "-o", LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("leaf_cap", C.c_int32),
                ("min_leaf_side", C.c_double), ("beta", C.c_double),
                ("min_vox_count", C.c_int32), ("rho_percentile", C.c_double),
                ("alpha", C.c_double), ("sigma", C.c_double),
                ("eps", C.c_double), ("keep_ratio", C.c_double),
                ("gamma", C.c_double), ("log_threshold", C.c_double),
                ("stages", C.c_int32)]


_P = C.c_void_p


class Out(C.Structure):
    _fields_ = [("key", _P), ("order", _P), ("leaf_of", _P), ("occ", _P),
                ("p1", _P), ("nbr_idx", _P), ("nbr_d2", _P), ("r2k", _P),
                ("rho", _P), ("p2", _P), ("score", _P), ("stage", _P),
                ("keep", _P), ("kept_idx", _P),
                ("leaf_begin", _P), ("leaf_end", _P), ("leaf_level", _P),
                ("leaf_prefix", _P), ("leaf_h", _P), ("leaf_n1", _P),
                ("leaf_n2", _P), ("leaf_m", _P), ("leaf_rho_med", _P),
                ("leaf_ncand", _P),
                ("n_kept", C.c_int64), ("n_leaves", C.c_int64),
                ("pairs", C.c_uint64), ("threads", C.c_int32)]


_lib = None


def _configure(h: C.CDLL) -> C.CDLL:
    h.orc_denoise.argtypes = [_P, C.c_int64, C.POINTER(Params), C.POINTER(Out)]
    h.orc_denoise.restype = C.c_int
    h.orc_default_params.argtypes = [C.POINTER(Params)]
    h.orc_morton_interleave.argtypes = [C.c_uint32] * 3
    h.orc_morton_interleave.restype = C.c_uint64
    h.orc_percentile_rank.argtypes = [C.c_int64, C.c_double]
    h.orc_percentile_rank.restype = C.c_int64
    h.orc_fit_loss_grad.argtypes = [_P, C.c_int64, C.c_int, C.c_double, C.POINTER(Out), _P,
                                    C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, _P]
    h.orc_fit_loss_grad.restype = C.c_int
    h.orc_nearest.argtypes = [_P, C.c_int64, _P, C.c_int64, _P, _P]
    h.orc_nearest.restype = C.c_int
    h.orc_eval_metrics.argtypes = [_P, C.c_int64, _P, C.c_int64, _P]
    h.orc_eval_metrics.restype = C.c_int
    return h


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _configure(C.CDLL(LIB_PATH))
    return _lib


def build_variant(source_text: str, out_path: str) -> C.CDLL:
    """Compile a modified copy of the oracle source (tests that plant a
    mistake in the oracle use this to show that a pin catches it) and load it.
    The regular library is left untouched."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    cmd = ["gcc", *CFLAGS, "-I", HERE, src, "-o", out_path, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return _configure(C.CDLL(out_path))


def default_params() -> dict:
    p = Params()
    lib().orc_default_params(C.byref(p))
    return {f: getattr(p, f) for f, _ in Params._fields_}


def morton(qx: int, qy: int, qz: int) -> int:
    return int(lib().orc_morton_interleave(qx, qy, qz))


def percentile_rank(n: int, q: float) -> int:
    return int(lib().orc_percentile_rank(n, q))


def denoise(xyz: np.ndarray, *, handle: C.CDLL | None = None, **params) -> dict:
    """Run the whole oracle pipeline; returns every intermediate array.

    ``handle`` selects another build of the oracle (``build_variant``); by
    default the regular library is used.

    Per-point arrays are in original point order. Rows of ``nbr_idx`` /
    ``nbr_d2`` / ``r2k`` / ``rho`` for points outside P1 are left at their
    fill values (0xFFFFFFFF / NaN).
    """
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    n = xyz.shape[0]
    p = default_params()
    unknown = set(params) - set(p)
    if unknown:
        raise TypeError(f"unknown parameters {sorted(unknown)}")
    p.update(params)
    P = Params(**p)
    k = P.k
    m = max(n, 1)
    a = dict(
        key=np.zeros(m, np.uint64), order=np.zeros(m, np.uint32),
        leaf_of=np.zeros(m, np.uint32), occ=np.zeros(m, np.uint32),
        p1=np.zeros(m, np.uint8),
        nbr_idx=np.full((m, k), 0xFFFFFFFF, np.uint32),
        nbr_d2=np.full((m, k), np.nan, np.float32),
        r2k=np.full(m, np.nan, np.float32), rho=np.full(m, np.nan, np.float64),
        p2=np.zeros(m, np.uint8), score=np.zeros(m, np.float64),
        stage=np.zeros(m, np.uint8), keep=np.zeros(m, np.uint8),
        kept_idx=np.zeros(m, np.uint32),
        leaf_begin=np.zeros(m, np.uint32), leaf_end=np.zeros(m, np.uint32),
        leaf_level=np.zeros(m, np.uint32), leaf_prefix=np.zeros(m, np.uint64),
        leaf_h=np.zeros(m, np.float32), leaf_n1=np.zeros(m, np.uint32),
        leaf_n2=np.zeros(m, np.uint32), leaf_m=np.zeros(m, np.uint32),
        leaf_rho_med=np.zeros(m, np.float64), leaf_ncand=np.zeros(m, np.uint32),
    )
    o = Out(**{name: arr.ctypes.data for name, arr in a.items()})
    h = lib() if handle is None else handle
    rc = h.orc_denoise(xyz.ctypes.data if n else None, n, C.byref(P), C.byref(o))
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    nl = o.n_leaves
    res = {}
    for name, arr in a.items():
        if name.startswith("leaf_") and name != "leaf_of":
            res[name] = arr[:nl].copy()
        elif name == "kept_idx":
            res[name] = arr[:o.n_kept].copy()
        else:
            res[name] = arr[:n].copy()
    res.update(n_kept=o.n_kept, n_leaves=nl, pairs=int(o.pairs),
               threads=o.threads, params=p)
    return res


def fit_loss_grad(xyz: np.ndarray, res: dict, label: np.ndarray, alpha: float, sigma: float, gamma: float,
                  tau: float, T: float) -> np.ndarray:
    """Score-fit loss and gradient (orc_fit_loss_grad) over the intermediates
    ``res`` of ``denoise(xyz, ...)``: [L, dL/dalpha, dL/dsigma, dL/dgamma,
    dL/dtau, number of terms]."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    n = xyz.shape[0]
    k = int(res["params"]["k"])
    keep = dict(nbr_idx=np.ascontiguousarray(res["nbr_idx"], np.uint32),
                rho=np.ascontiguousarray(res["rho"], np.float64),
                p2=np.ascontiguousarray(res["p2"], np.uint8),
                leaf_of=np.ascontiguousarray(res["leaf_of"], np.uint32),
                leaf_rho_med=np.ascontiguousarray(res["leaf_rho_med"], np.float64))
    o = Out(**{name: arr.ctypes.data for name, arr in keep.items()})
    lab = np.ascontiguousarray(label, np.uint8)
    out = np.zeros(6, np.float64)
    rc = lib().orc_fit_loss_grad(xyz.ctypes.data, n, k, float(res["params"]["eps"]), C.byref(o), lab.ctypes.data,
                                 alpha, sigma, gamma, tau, T, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle rejected the fit parameters")
    return out


def nearest(a: np.ndarray, b: np.ndarray):
    """Nearest point of b for every point of a: (idx uint32, fp32 d2)."""
    a = np.ascontiguousarray(a, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    idx = np.zeros(max(len(a), 1), np.uint32)
    d2 = np.zeros(max(len(a), 1), np.float32)
    if lib().orc_nearest(a.ctypes.data, len(a), b.ctypes.data, len(b), idx.ctypes.data, d2.ctypes.data) != 0:
        raise ValueError("empty reference set")
    return idx[:len(a)], d2[:len(a)]


def eval_metrics(clean: np.ndarray, den: np.ndarray) -> np.ndarray:
    """[MSE, mean denoised->clean, CD (Eq. 30), PSNR dB (Eq. 29)]."""
    clean = np.ascontiguousarray(clean, np.float32)
    den = np.ascontiguousarray(den, np.float32)
    out = np.zeros(4, np.float64)
    if lib().orc_eval_metrics(clean.ctypes.data, len(clean), den.ctypes.data, len(den), out.ctypes.data) != 0:
        raise ValueError("empty cloud")
    return out
