"""Second-stage rescoring of the ranked poses (the method's fourth step) on the GPU, through the
C ABI, against the FP64 oracle: every ranked pose's second-stage score equals the oracle's score
of the pose its descriptor names (FP64 on both sides: 1e-9 relative), the chosen pose is the
lowest of the list (ties to the earlier entry), and a persistent launch replayed from a graph
gives the same scores bit for bit as one launch per pocket."""
import sys

import numpy as np
import pytest

import exs_synth as S
from parity import gpu_desc_to_theta_tau

pytestmark = pytest.mark.gpu

KEEP = 30


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


def run(B, pockets, batch, s, flags=0, lpw=0):
    pids = [B.exs_load_pocket_grid(p.values, p.spacing, p.origin) for p in pockets]
    try:
        bid = B.exs_upload_ligands(batch, pocket_ids=pids)
        prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                              s.clash_cutoff, s.clash_penalty, ligands_per_wg=lpw,
                              flags=flags | B.EXS_FLAG_RESCORE2, cluster_rmsd_A=3.0,
                              rank_keep=KEEP)
        job = B.exs_dock_batch(bid, prm)
        L = batch.n_ligands
        r2 = B.exs_get_rescored_poses(job, L, KEEP)
        _, ranked = B.exs_get_ranked_poses(job, L, KEEP)
        orient = B.exs_get_orientation_results(job, L, s.n_orient)
        B.exs_release_job(job)
        B.exs_release_ligands(bid)
    finally:
        for pid in pids:
            B.exs_unload_pocket(pid)
    return r2, ranked, orient


def check(O, grids, s, batch, r2, ranked, orient):
    prm = O.Params.of(s)
    worst, decided = 0.0, 0
    for l in range(batch.n_ligands):
        lig = batch.ligand(l)
        ref = []
        for t in range(KEEP):
            k = int(ranked[l, t])
            th, ta = gpu_desc_to_theta_tau(orient["desc"][l, k], len(lig.rot))
            X = O.pose_from_desc(grids[lig.pocket], prm, lig, k, th, ta)
            e, _ = O.rescore2(grids[lig.pocket], lig, X, sigma=s.clash_cutoff)
            got = float(r2["score2"][l, t])
            assert abs(got - e) <= 1e-9 * max(1.0, abs(e)), (l, t, got, e)
            worst = max(worst, abs(got - e) / max(1.0, abs(e)))
            ref.append(e)
        sc = r2["score2"][l]
        j = O.stage2_best(sc)
        assert int(r2["best_orient"][l]) == int(ranked[l, j])
        assert float(r2["best_score2"][l]) == float(sc[j])
        jo = O.stage2_best(ref)
        srt = sorted(ref)
        if srt[1] - srt[0] > 1e-9 * max(1.0, abs(srt[0])):   # the oracle's choice is clear-cut
            assert jo == j, (l, jo, j)
            decided += 1
    return worst, decided


def test_rescored_poses_match_oracle(B, oracle_lib):
    O = oracle_lib
    p = S.make_pocket("small")
    batch = S.make_ligand_batch("small", 0, 16)
    s = S.SearchSettings(64, 16, 1, 27)
    log("second-stage rescoring: 16 ligands, K=64, keep %d" % KEEP)
    r2, ranked, orient = run(B, [p], batch, s)
    worst, decided = check(O, [O.Grid.of(p)], s, batch, r2, ranked, orient)
    log("max relative error %.3g, oracle choice clear-cut on %d ligands" % (worst, decided))
    assert decided >= batch.n_ligands // 2


def test_rescoring_of_the_largest_ligands(B, oracle_lib):
    """Two atoms per lane: ligands of 64, 65, 101 and 128 atoms (even and odd counts, so that
    every rule of the pair split over the atoms is taken) and up to 32 rotatable bonds; every
    ranked pose's second-stage score matches the oracle's."""
    O = oracle_lib
    p = S.make_pocket("small")
    ligs = []
    for i, (n, nrot) in enumerate(((64, 6), (65, 9), (101, 20), (128, 32))):
        wl = S.Workload("big%d" % n, 100 + i, 1, 1, (48,), 0.5, 4, ("fixed", n), ("fixed", nrot),
                        S.SearchSettings(64, 8, 1, 27))
        ligs += S.make_ligands(wl, 0, 1)
    batch = S.batch_from_ligands(ligs)
    s = S.SearchSettings(64, 8, 1, 27)
    log("second-stage rescoring of n=%s" % [l.n for l in ligs])
    r2, ranked, orient = run(B, [p], batch, s)
    worst, decided = check(O, [O.Grid.of(p)], s, batch, r2, ranked, orient)
    log("max relative error %.3g, oracle choice clear-cut on %d ligands" % (worst, decided))


def test_rescoring_persistent_graph_equals_per_pocket(B, oracle_lib):
    """Uneven ligands over two pockets, up to 15 rotatable bonds: one persistent launch replayed
    from a hipGraph equals the per-pocket launches bit for bit, and a sample matches the oracle."""
    O = oracle_lib
    wl = S.Workload("mixed2", 93, 24, 2, (32, 40), 0.375, 8, ("lognormal", 35.0, 0.4, 10, 90),
                    ("uniform", 0, 15), S.SearchSettings(64, 8, 1, 27))
    pockets = [S.make_pocket(wl, i) for i in range(2)]
    batch = S.make_ligand_batch(wl, 0, 24)
    a = run(B, pockets, batch, wl.search)
    for rep in range(2):
        b = run(B, pockets, batch, wl.search, flags=B.EXS_FLAG_PERSISTENT | B.EXS_FLAG_GRAPH, lpw=1)
        for key in ("score2", "best_orient", "best_score2"):
            assert np.array_equal(a[0][key], b[0][key]), (rep, key)
        assert np.array_equal(a[1], b[1])
    sub = list(range(0, 24, 3))
    r2 = {k: v[sub] for k, v in a[0].items()}
    orient = {k: v[sub] for k, v in a[2].items()}
    check(O, [O.Grid.of(pk) for pk in pockets], wl.search, batch.subset(sub), r2, a[1][sub], orient)


def test_rescoring_request_errors(B):
    p = S.make_pocket("small")
    batch = S.make_ligand_batch("small", 0, 2)
    pid = B.exs_load_pocket_grid(p.values, p.spacing, p.origin)
    try:
        bid = B.exs_upload_ligands(batch, pocket_ids=[pid])
        with pytest.raises(B.ExsError) as ei:       # rescoring needs the ranked list
            B.exs_dock_batch(bid, B.search_params(8, 8, 1, 1, flags=B.EXS_FLAG_RESCORE2))
        assert ei.value.code == B.EXS_EINVAL
        job = B.exs_dock_batch(bid, B.search_params(8, 8, 1, 1, rank_keep=4))
        with pytest.raises(B.ExsError) as ei:       # the job did not rescore
            B.exs_get_rescored_poses(job, 2, 4)
        assert ei.value.code == B.EXS_EINVAL
        B.exs_release_job(job)
        B.exs_release_ligands(bid)
    finally:
        B.exs_unload_pocket(pid)


def test_job_stage_times(B):
    """exs_job_stage_ms: an eager job that ranks and rescores reports the time of each step,
    positive and adding up to the job's time; a job that ranks without rescoring reads -1 for
    the rescoring, and a job without ranking gives its whole time as the search."""
    p = S.make_pocket("small")
    batch = S.make_ligand_batch("small", 0, 16)
    pid = B.exs_load_pocket_grid(p.values, p.spacing, p.origin)
    bid = None
    try:
        bid = B.exs_upload_ligands(batch, pocket_ids=[pid])
        for flags, keep in ((B.EXS_FLAG_RESCORE2, KEEP), (0, KEEP), (0, 0)):
            prm = B.search_params(64, 16, 1, 27, flags=flags, cluster_rmsd_A=3.0, rank_keep=keep)
            job = B.exs_dock_batch(bid, prm)
            st = B.exs_job_stage_ms(job)
            tot = B.exs_job_elapsed_ms(job)
            B.exs_release_job(job)
            log("stages", flags, keep, st, tot)
            assert st["dock"] > 0
            if keep:
                assert st["rank"] > 0
            else:
                assert st["rank"] == -1 and st["rescore2"] == -1
            if flags:
                assert st["rescore2"] > 0
            elif keep:
                assert st["rescore2"] == -1
            parts = st["dock"] + max(st["rank"], 0.0) + max(st["rescore2"], 0.0)
            assert abs(parts - tot) <= 1e-3 + 1e-3 * tot, (parts, tot)
    finally:
        if bid is not None:
            B.exs_release_ligands(bid)
        B.exs_unload_pocket(pid)
