"""GPU ranking of each ligand's final poses (Sec. 3.1, third step) against the FP64 oracle.

Per ligand the oracle docks the ligand itself (FP64 final poses and scores) and ranks those
poses.  Where the GPU followed the oracle's trajectory in every orientation and the oracle
flags no RMSD within 1e-4 A of the threshold and no pair of adjacent scores closer than the
score tolerance, the GPU's cluster count and ranked list must equal the oracle's exactly.
Otherwise the GPU list must be a valid ranking of the poses the GPU found (rebuilt in FP64 by
the oracle from the GPU descriptors): leaders first, each group by score within tolerance,
every leader at least thr - 1e-4 A from every better leader, every other pose within
thr + 1e-4 A of a better-or-equal leader."""
import sys

import numpy as np
import pytest

import exs_synth as S
from parity import tol

pytestmark = pytest.mark.gpu
DELTA = 1e-4


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2110_11644_amd import binding
    binding.lib()
    return binding


def run_ranked(B, pocket, batch, s, thr, keep, flags=0, lpw=0):
    pid = B.exs_load_pocket_grid(pocket.values, pocket.spacing, pocket.origin)
    try:
        bid = B.exs_upload_ligands(batch, pocket_ids=[pid])
        prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                              s.clash_cutoff, s.clash_penalty, flags=flags, ligands_per_wg=lpw,
                              cluster_rmsd_A=thr, rank_keep=keep)
        job = B.exs_dock_batch(bid, prm)
        nc, rk = B.exs_get_ranked_poses(job, batch.n_ligands, keep)
        orient = B.exs_get_orientation_results(job, batch.n_ligands, s.n_orient)
        B.exs_release_job(job)
        B.exs_release_ligands(bid)
    finally:
        B.exs_unload_pocket(pid)
    return nc, rk, orient


def valid_ranking(O, poses, scores, ranked, n_lead, thr):
    lead, rest = list(ranked[:n_lead]), list(ranked[n_lead:])
    for grp in (lead, rest):
        for a, b in zip(grp, grp[1:]):
            assert scores[a] <= scores[b] + tol(scores[b]), "group not sorted by score"
    for i, k in enumerate(lead):
        for q in lead[:i]:
            assert O.rmsd(poses[k], poses[q]) >= thr - DELTA, "leaders %d and %d are similar" % (q, k)
    for k in rest:
        ok = any(O.rmsd(poses[k], poses[q]) < thr + DELTA and scores[q] <= scores[k] + tol(scores[k])
                 for q in lead)
        assert ok, "pose %d has no better leader within the threshold" % k


def check_ranking(O, grid, prm, batch, nc, rk, orient, thr, keep, stats):
    K = prm.n_orient
    for l in range(batch.n_ligands):
        lig = batch.ligand(l)
        nrot = len(lig.rot)
        ref = O.dock_ligand(grid, prm, lig, coords=True)
        desc = orient["desc"][l]
        same = all(np.array_equal(np.asarray(desc[k]["theta"][:nrot], np.int64) % prm.torsion_steps,
                                  ref["theta"][k] % prm.torsion_steps)
                   and np.array_equal(np.asarray(desc[k]["tau"], np.int64), ref["tau"][k])
                   for k in range(K))
        r = O.rank_poses(ref["coords"], ref["score"], thr, DELTA, 1e-4)
        n_lead = int(nc[l])
        assert 1 <= n_lead <= K
        if same and r["amb_rmsd"] == 0 and r["amb_score"] == 0:
            assert n_lead == r["n_leaders"], "ligand %d: %d clusters vs oracle %d" % (
                l, n_lead, r["n_leaders"])
            assert rk[l].tolist() == r["order"][:keep].tolist(), "ligand %d: ranked list differs" % l
            stats["exact"] = stats.get("exact", 0) + 1
        else:
            assert keep == K, "ambiguous ligand needs the full list to be checked"
            assert sorted(rk[l].tolist()) == list(range(K))
            poses = np.stack([O.pose_from_desc(grid, prm, lig, k,
                                               np.asarray(desc[k]["theta"][:nrot], np.int64),
                                               np.asarray(desc[k]["tau"], np.int64))
                              for k in range(K)])
            valid_ranking(O, poses, orient["score"][l].astype(np.float64), rk[l], n_lead, thr)
            stats["valid"] = stats.get("valid", 0) + 1
        stats["clusters"] = stats.get("clusters", 0) + n_lead


@pytest.mark.parametrize("thr", [3.0, 1.0], ids=["3A", "1A"])
def test_ranked_poses_match_oracle(B, oracle_lib, thr):
    O = oracle_lib
    pocket = S.make_pocket("small")
    batch = S.make_ligand_batch("small").subset(range(24))
    s = S.SMALL.search
    K = s.n_orient
    log("ranking: 24 ligands x 64 orientations, thr %.1f A" % thr)
    nc, rk, orient = run_ranked(B, pocket, batch, s, thr, K)
    stats = {}
    check_ranking(O, O.Grid.of(pocket), O.Params.of(s), batch, nc, rk, orient, thr, K, stats)
    log("ranking stats", stats)
    assert stats.get("exact", 0) >= batch.n_ligands // 2
    # keeping the first 30 (as the paper rescored) truncates the same list
    nc30, rk30, _ = run_ranked(B, pocket, batch, s, thr, 30)
    assert np.array_equal(nc30, nc) and np.array_equal(rk30, rk[:, :30])


def test_ranking_with_offsets_and_persistent_launch(B, oracle_lib):
    """T = 27 offsets, K = 100 (not a multiple of 64), persistent launch with two ligands per
    workgroup: the ranking still matches the oracle."""
    O = oracle_lib
    pocket = S.make_pocket("small")
    batch = S.make_ligand_batch("small").subset(range(8))
    s = S.SearchSettings(100, 16, 1, 27)
    nc, rk, orient = run_ranked(B, pocket, batch, s, 3.0, 100, flags=B.EXS_FLAG_PERSISTENT, lpw=2)
    stats = {}
    check_ranking(O, O.Grid.of(pocket), O.Params.of(s), batch, nc, rk, orient, 3.0, 100, stats)
    log("ranking (T=27, K=100) stats", stats)


def test_ranking_of_the_largest_ligands(B, oracle_lib):
    """Ligands of 64, 65, 101 and 128 atoms (pose rows in whole batches of 8 and with a tail)
    and up to 32 rotatable bonds: the ranking matches the oracle."""
    O = oracle_lib
    pocket = S.make_pocket("small")
    ligs = []
    for i, (n, nrot) in enumerate(((64, 6), (65, 9), (101, 20), (128, 32))):
        wl = S.Workload("big%d" % n, 96 + i, 1, 1, (48,), 0.5, 4, ("fixed", n), ("fixed", nrot),
                        S.SMALL.search)
        ligs += S.make_ligands(wl, 0, 1)
    batch = S.batch_from_ligands(ligs)
    s = S.SMALL.search
    nc, rk, orient = run_ranked(B, pocket, batch, s, 3.0, s.n_orient)
    stats = {}
    check_ranking(O, O.Grid.of(pocket), O.Params.of(s), batch, nc, rk, orient, 3.0, s.n_orient, stats)
    log("ranking (n = 64-128) stats", stats)


def test_ranking_request_errors(B):
    pocket = S.make_pocket("small")
    batch = S.make_ligand_batch("small").subset(range(2))
    pid = B.exs_load_pocket_grid(pocket.values, pocket.spacing, pocket.origin)
    try:
        bid = B.exs_upload_ligands(batch, pocket_ids=[pid])
        with pytest.raises(B.ExsError) as ei:
            B.exs_dock_batch(bid, B.search_params(8, 8, 1, 1, rank_keep=9))
        assert ei.value.code == B.EXS_EINVAL
        with pytest.raises(B.ExsError) as ei:
            B.exs_dock_batch(bid, B.search_params(8, 8, 1, 1, rank_keep=4, cluster_rmsd_A=float("nan")))
        assert ei.value.code == B.EXS_EINVAL
        job = B.exs_dock_batch(bid, B.search_params(8, 8, 1, 1))
        with pytest.raises(B.ExsError) as ei:
            B.exs_get_ranked_poses(job, 2, 4)
        assert ei.value.code == B.EXS_EINVAL
        B.exs_release_job(job)
        B.exs_release_ligands(bid)
    finally:
        B.exs_unload_pocket(pid)
