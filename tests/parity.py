"""GPU-vs-oracle acceptance helpers (test infrastructure).

Acceptance of a GPU docking result against the FP64 oracle, with
tol(s) = 1e-4 * max(|s|, 1) (relative per-pose score tolerance of the FP32 path):

1. per pose     every orientation's GPU score matches the oracle's FP64 score of
                the pose the GPU descriptor names, within tol plus one penalty per
                clash pair whose distance is within the ambiguity band;
2. trajectory   GPU descriptor == oracle descriptor, except on orientations the
                oracle flags as near ties (a decision whose gap is below tol);
3. best pose    the GPU best score equals the oracle best within tol, unless the
                difference is explained by near-tie orientations (ties accepted);
                the GPU's best orientation is the argmin of its own scores;
4. RMSD         the GPU best-pose coordinates match the oracle's rebuild of the
                GPU descriptor within 0.01 A (no superposition).
"""
from __future__ import annotations

import numpy as np

REL_TOL = 1e-4
RMSD_TOL = 0.01


def tol(s: float) -> float:
    return REL_TOL * max(abs(s), 1.0)


def gpu_desc_to_theta_tau(desc_row, nrot):
    theta = np.asarray(desc_row["theta"][:nrot], dtype=np.int64)
    tau = np.asarray(desc_row["tau"], dtype=np.int64)
    return theta, tau


def check_ligand(O, grid, prm, lig, gpu_scores, gpu_desc, best_score, best_desc, best_xyz,
                 ref=None, stats=None):
    """Check one ligand; raises AssertionError with a message on failure.

    gpu_scores [K], gpu_desc [K] (POSE_DESC rows), best_* from exs_get_best_poses.
    """
    K = prm.n_orient
    nrot = len(lig.rot)
    if ref is None:
        ref = O.dock_ligand(grid, prm, lig)
    stats = stats if stats is not None else {}
    # 1. per pose
    worst = 0.0
    for k in range(K):
        th, ta = gpu_desc_to_theta_tau(gpu_desc[k], nrot)
        assert int(gpu_desc[k]["orient"]) == k
        e, _, amb = O.rescore_desc(grid, prm, lig, k, th, ta)[:3]
        err = abs(float(gpu_scores[k]) - e)
        allow = tol(e) + prm.clash_penalty * amb
        assert err <= allow, "pose %d: gpu %.7g vs oracle(desc) %.7g (amb %d)" % (
            k, gpu_scores[k], e, amb)
        worst = max(worst, err / max(abs(e), 1.0))
    stats["max_rel_err"] = max(stats.get("max_rel_err", 0.0), worst)
    # 2. trajectory
    near = ref["near_tie"]
    mism = 0
    for k in range(K):
        th, ta = gpu_desc_to_theta_tau(gpu_desc[k], nrot)
        same = (np.array_equal(th % prm.torsion_steps, ref["theta"][k] % prm.torsion_steps)
                and np.array_equal(ta, ref["tau"][k]))
        if not same:
            assert near[k], "orientation %d: trajectory differs and the oracle saw no near tie" % k
            mism += 1
    stats["near_tie"] = stats.get("near_tie", 0) + int(near.sum())
    stats["diverged_on_near_tie"] = stats.get("diverged_on_near_tie", 0) + mism
    stats["orientations"] = stats.get("orientations", 0) + K
    # 3. best pose
    g = np.asarray(gpu_scores, dtype=np.float64)
    kg = int(np.argmin(g))            # first minimum = lowest orientation among ties
    assert int(best_desc["orient"]) == kg, "best orientation %d is not the argmin %d" % (
        int(best_desc["orient"]), kg)
    assert float(best_score) == float(g[kg])
    r = ref["score"]
    kr = int(ref["best_k"])
    if abs(g[kg] - r[kr]) > tol(r[kr]):
        assert near[kg] or near[kr], "best %.7g (k=%d) vs oracle %.7g (k=%d), no near tie" % (
            g[kg], kg, r[kr], kr)
        stats["best_tie_accepted"] = stats.get("best_tie_accepted", 0) + 1
    # 4. RMSD of the best pose (best_xyz None: the caller checks the coordinates itself)
    if best_xyz is None:
        return stats
    th, ta = gpu_desc_to_theta_tau(best_desc, nrot)
    X = O.pose_from_desc(grid, prm, lig, kg, th, ta)
    rmsd = float(np.sqrt(np.mean(np.sum((np.asarray(best_xyz, np.float64) - X) ** 2, axis=1))))
    assert rmsd <= RMSD_TOL, "best-pose RMSD %.4g A" % rmsd
    stats["max_rmsd"] = max(stats.get("max_rmsd", 0.0), rmsd)
    return stats


def check_best_pose(O, grid, prm, lig, best_score, best_desc, best_xyz, ref=None):
    """Best pose only (results that carry no per-orientation scores, e.g. served requests):
    the GPU score is the oracle's FP64 score of the GPU descriptor within tol (+ ambiguous
    pairs); it equals the oracle's best within tol unless a near tie explains the difference;
    the coordinates are the descriptor's pose within RMSD_TOL.  Returns the oracle result."""
    nrot = len(lig.rot)
    th, ta = gpu_desc_to_theta_tau(best_desc, nrot)
    k = int(best_desc["orient"])
    e, _, amb, X = O.rescore_desc(grid, prm, lig, k, th, ta)
    assert abs(float(best_score) - e) <= tol(e) + prm.clash_penalty * amb, (
        "best pose: gpu %.7g vs oracle(desc) %.7g (amb %d)" % (best_score, e, amb))
    if ref is None:
        ref = O.dock_ligand(grid, prm, lig)
    kr = int(ref["best_k"])
    if abs(float(best_score) - ref["best_score"]) > tol(ref["best_score"]):
        assert ref["near_tie"][k] or ref["near_tie"][kr], (
            "best %.7g (k=%d) vs oracle %.7g (k=%d), no near tie" % (best_score, k,
                                                                   ref["best_score"], kr))
    rmsd = float(np.sqrt(np.mean(np.sum((np.asarray(best_xyz, np.float64) - X) ** 2, axis=1))))
    assert rmsd <= RMSD_TOL, "best-pose RMSD %.4g A" % rmsd
    return ref


def oracle_topk_fp64_best(O, grid_search, grid_master, prm, lig, top_k, ref=None):
    """The oracle's own run of the mixed-precision path: its search on the grid the GPU searched
    (e.g. the RNE-rounded 16-bit grid), its top_k orientations by (score, k), each rescored in
    FP64 on the FP32 master grid, and the best of those.  Returns (best64, k, ambiguous) where
    `ambiguous` is set when the selection is not decided beyond the FP32 tolerance: a near tie
    in a top_k trajectory, top_k-th and next scores within tol, or two rescored scores within
    tol of the best."""
    if ref is None:
        ref = O.dock_ligand(grid_search, prm, lig)
    sc = ref["score"]
    K = len(sc)
    order = sorted(range(K), key=lambda k: (sc[k], k))
    tk = min(top_k, K)
    top = order[:tk]
    e64 = []
    for k in top:
        e = O.rescore_desc(grid_master, prm, lig, k, ref["theta"][k], ref["tau"][k])[0]
        e64.append(e)
    j = int(np.argmin(e64))
    amb = bool(any(ref["near_tie"][k] for k in top))
    if tk < K and abs(sc[order[tk]] - sc[order[tk - 1]]) <= tol(sc[order[tk - 1]]):
        amb = True
    srt = sorted(e64)
    if len(srt) > 1 and srt[1] - srt[0] <= tol(srt[0]):
        amb = True
    return float(e64[j]), int(top[j]), amb
