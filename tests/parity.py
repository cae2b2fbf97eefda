"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI,
pull every intermediate back, and compare it with the oracle element by element.
"""
import numpy as np

SCORE_RTOL = 1e-5  # scores vs the FP64 oracle (relative), keep-label tolerance band


def run_gpu(den, xyz):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(xyz, np.float32)).cuda()
    res = den(x)
    n = xyz.shape[0]
    out = {}
    torch.cuda.synchronize()
    out["keep"] = res.keep.cpu().numpy()
    out["score"] = res.score.cpu().numpy()
    out["stage"] = res.stage.cpu().numpy()
    out["n_kept"] = int(res.n_kept.cpu().item())
    out["kept_idx"] = res.kept_idx.cpu().numpy().view(np.uint32)[:out["n_kept"]]
    if n == 0:
        return out
    counts = den.dump("COUNTS", n).cpu().numpy()
    out["n_leaves"], out["n_p1"], out["pairs"], _ = [int(c) for c in counts]
    out["status"] = int(den.dump("STATUS", n).cpu().numpy()[0])
    nl = out["n_leaves"]
    u32 = lambda t: t.cpu().numpy().view(np.uint32)
    out["key"] = den.dump("KEYS", n).cpu().numpy().view(np.uint64)
    out["order"] = u32(den.dump("ORDER", n))
    out["leaf_of"] = u32(den.dump("LEAF_OF", n))
    lt = u32(den.dump("LEAF_TABLE", n))[:nl]
    out["leaf_begin"], out["leaf_end"], out["leaf_level"] = lt[:, 0], lt[:, 1], lt[:, 2]
    out["leaf_h"] = lt[:, 3].copy().view(np.float32)
    out["occ"] = u32(den.dump("OCC", n))
    out["p1"] = den.dump("P1", n).cpu().numpy()
    out["nbr_idx"] = u32(den.dump("NBR_IDX", n))
    out["nbr_d2"] = den.dump("NBR_D2", n).cpu().numpy()
    out["r2k"] = den.dump("R2K", n).cpu().numpy()
    out["rho"] = den.dump("RHO", n).cpu().numpy()
    out["p2"] = den.dump("P2", n).cpu().numpy()
    out["leaf_rho_med"] = den.dump("LEAF_RHO_MED", n).cpu().numpy()[:nl]
    out["score64"] = den.dump("SCORE64", n).cpu().numpy()
    out["leaf_ncand"] = u32(den.dump("LEAF_NCAND", n))[:nl]
    return out


SHORT_SORT_LEVEL = 10  # the radix passes cover key bits 32..62 (every level-10 prefix)


def expected_order(ref):
    """The kernels' sorted order: (key bits 32..62, original index), except
    inside "deep" level-10 cells (more than leaf_cap points, split further by
    the octree) and the level-10 cells next to them (where the deep leaves'
    halo cells reach), which are re-sorted on the whole key: there the order
    is the oracle's (key, index). Deep cells exist exactly when a leaf lies
    below level 10."""
    n = len(ref["keep"])
    key = ref["key"].astype(np.uint64)
    masked = key & ~np.uint64(0xFFFFFFFF)
    if ref["n_leaves"] and int(ref["leaf_level"].max()) > SHORT_SORT_LEVEL:
        cell = key >> np.uint64(3 * (21 - SHORT_SORT_LEVEL))
        u, cnt = np.unique(cell, return_counts=True)
        resort = set()
        side = 1 << SHORT_SORT_LEVEL
        for c in u[cnt > int(ref["params"]["leaf_cap"])]:
            c = int(c)
            xyz = [sum(((c >> (3 * b + a)) & 1) << b for b in range(SHORT_SORT_LEVEL)) for a in range(3)]
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        q = (xyz[0] + dx, xyz[1] + dy, xyz[2] + dz)
                        if min(q) < 0 or max(q) >= side:
                            continue
                        resort.add(sum(((q[a] >> b) & 1) << (3 * b + a)
                                       for b in range(SHORT_SORT_LEVEL) for a in range(3)))
        full = np.isin(cell, np.array(sorted(resort), np.uint64))
        masked = np.where(full, key, masked)
    return np.lexsort((np.arange(n), masked)).astype(np.uint32)


def check_order(order, ref, expect=None):
    """The sorted order is exactly the one above; every leaf's points fill its
    range [begin, end) in leaf order. expect = "full" additionally requires the
    oracle's whole-key order (every point in a deep cell or alone in its
    level-10 cell), "short" that no cell was re-sorted."""
    n = len(ref["keep"])
    assert np.array_equal(np.sort(order), np.arange(n, dtype=order.dtype)), "order is not a permutation"
    sizes = (ref["leaf_end"] - ref["leaf_begin"]).astype(np.int64)
    want = np.repeat(np.arange(ref["n_leaves"], dtype=np.uint32), sizes)
    assert np.array_equal(ref["leaf_of"][order], want), "order: a point outside its leaf's range"
    exp = expected_order(ref)
    assert np.array_equal(order, exp), "order: not (key bits 32..62, index) with deep cells in key order"
    if expect == "full":
        assert np.array_equal(order, ref["order"]), "order: expected the full key order"
    elif expect == "short":
        assert int(ref["leaf_level"].max()) <= SHORT_SORT_LEVEL, "order: a deep cell where none was expected"


def leaf_thresholds(ref):
    """theta_t: the smallest oracle score kept in each leaf (inf if none)."""
    th = np.full(ref["n_leaves"], np.inf)
    kept = np.nonzero(ref["keep"])[0]
    if len(kept):
        np.minimum.at(th, ref["leaf_of"][kept], ref["score"][kept])
    return th


def compare(g, ref, exact_rho=False, log_threshold=None, order=None):
    """Assert GPU results match the oracle to the parity bar; return stats.
    With log_threshold (threshold keep mode) the cut is e^threshold in every leaf."""
    n = len(ref["keep"])
    stats = {}
    if n == 0:
        assert g["n_kept"] == 0
        return stats
    assert g["status"] == 0, f"device status {g['status']}"
    assert g["n_leaves"] == ref["n_leaves"]
    for f in ["key", "leaf_of", "occ", "p1"]:
        assert np.array_equal(g[f], ref[f]), f
    for f in ["leaf_begin", "leaf_end", "leaf_level", "leaf_ncand"]:
        assert np.array_equal(g[f], ref[f]), f
    check_order(g["order"], ref, order)
    assert np.array_equal(g["leaf_h"].view(np.uint32), ref["leaf_h"].view(np.uint32)), "leaf_h"
    assert g["n_p1"] == int(ref["p1"].sum())
    assert g["pairs"] == ref["pairs"]
    p1 = ref["p1"] == 1
    assert np.array_equal(g["nbr_idx"][p1], ref["nbr_idx"][p1]), "nbr_idx"
    assert np.array_equal(g["nbr_d2"][p1].view(np.uint32), ref["nbr_d2"][p1].view(np.uint32)), "nbr_d2"
    assert np.array_equal(g["r2k"][p1].view(np.uint32), ref["r2k"][p1].view(np.uint32)), "r2k"
    assert np.array_equal(g["p2"], ref["p2"]), "p2"
    # density and median: FP64, same expressions on both sides
    r_ref, r_gpu = ref["rho"][p1], g["rho"][p1]
    fin = np.isfinite(r_ref)
    assert np.array_equal(np.isfinite(r_gpu), fin)
    if fin.any():
        rel = np.abs(r_gpu[fin] - r_ref[fin]) / np.maximum(np.abs(r_ref[fin]), 1e-300)
        stats["rho_max_rel"] = float(rel.max())
        assert rel.max() <= 1e-12
    m_ref, m_gpu = ref["leaf_rho_med"], g["leaf_rho_med"]
    finm = np.isfinite(m_ref)
    assert np.allclose(m_gpu[finm], m_ref[finm], rtol=1e-12, atol=0)
    # scores: FP64 on the GPU, checked to the stated relative tolerance
    s2 = ref["p2"] == 1
    assert np.array_equal(g["score64"] >= 0, ref["score"] >= 0)
    F = ref["score"][s2]
    Fg = g["score64"][s2]
    both_nan = np.isnan(F) & np.isnan(Fg)
    both_inf = np.isinf(F) & np.isinf(Fg)
    ok = both_nan | both_inf | (np.abs(Fg - F) <= SCORE_RTOL * np.abs(F))
    assert ok.all(), f"score64 mismatches: {np.count_nonzero(~ok)}"
    finF = np.isfinite(F) & (F != 0)
    if finF.any():
        stats["score_max_rel"] = float((np.abs(Fg - F)[finF] / np.abs(F[finF])).max())
    F32 = g["score"][s2]
    ok32 = both_nan | both_inf | (np.abs(F32 - F) <= SCORE_RTOL * np.abs(F))
    assert ok32.all(), "score (fp32 output)"
    assert np.all(g["score"][~s2] == -1.0)
    # labels: may differ only within the tolerance band around the leaf threshold
    th = leaf_thresholds(ref) if log_threshold is None else np.full(ref["n_leaves"], np.exp(log_threshold))
    diff = np.nonzero(g["keep"] != ref["keep"])[0]
    for i in diff:
        t = ref["leaf_of"][i]
        assert ref["p2"][i] == 1, f"label differs outside P2 at {i}"
        assert abs(ref["score"][i] - th[t]) <= SCORE_RTOL * th[t], f"label differs at {i}"
    stats["label_diffs"] = int(len(diff))
    # stage codes agree wherever the label does
    same = g["keep"] == ref["keep"]
    assert np.array_equal(g["stage"][same], ref["stage"][same])
    # compaction
    assert g["n_kept"] == int(g["keep"].sum())
    assert np.array_equal(g["kept_idx"], np.nonzero(g["keep"])[0].astype(np.uint32))
    return stats
