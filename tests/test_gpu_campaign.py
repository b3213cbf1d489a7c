"""Screening campaign on the GPU (exs_campaign_run: a host library streamed in chunks through
the serving engine by packer threads, hits merged) against one plain launch and the FP64
oracle: every ligand's best score equals the plain launch's bit for bit, the plain launch's
best poses pass the best-pose acceptance against the oracle, and the hit list is the oracle's
except for ligands within the score tolerance of the cut."""
import sys

import numpy as np
import pytest

import exs_synth as S
from parity import check_best_pose, tol

pytestmark = pytest.mark.gpu

WL = S.Workload("campaign-test", 94, 0, 3, (32, 40, 48), 0.375, 8, ("lognormal", 35.0, 0.4, 10, 90),
                ("uniform", 0, 15), S.SearchSettings(64, 8, 1, 27))


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


def test_campaign_hits_match_oracle(B, oracle_lib):
    O = oracle_lib
    s = WL.search
    pockets = [S.make_pocket(WL, i) for i in range(3)]
    ligs = S.make_ligands(WL, 0, 400)
    rng = np.random.default_rng(17)
    for l in ligs:
        l.pocket = int(rng.integers(0, 3))
    library = S.batch_from_ligands(ligs)
    L, A = library.n_ligands, int(library.atom_offset[-1])
    prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, poses_per_lane=1,
                          ligands_per_wg=1, flags=B.EXS_FLAG_PERSISTENT)
    pids = [B.exs_load_pocket_grid(p.values, p.spacing, p.origin) for p in pockets]
    try:
        log("campaign: 400 ligands, chunks of 64, 3 packers, top 5 %")
        res = B.exs_campaign_run(pids, prm, library, chunk_ligands=64, packers=3,
                                 hit_fraction=0.05, library_pocket_ids=pids)
        bid = B.exs_upload_ligands(library, pocket_ids=pids)
        job = B.exs_dock_batch(bid, B.search_params(s.n_orient, s.torsion_steps, s.passes,
                                                    s.n_offsets))
        plain = B.exs_get_best_poses(job, L, A)
        B.exs_release_job(job)
        B.exs_release_ligands(bid)
        with pytest.raises(B.ExsError) as ei:          # an invalid ligand: nothing is docked
            bad = library.subset(range(8))
            bad.type[3] = 9
            B.exs_campaign_run(pids, prm, bad, library_pocket_ids=pids)
        assert ei.value.code == B.EXS_EINVAL
    finally:
        for pid in pids:
            B.exs_unload_pocket(pid)
    st = res["stats"]
    log("stats", st)
    assert st["ligands"] == L and st["chunks"] == 7 and st["hits"] == 20
    # the validation pass and the first submission happen within the call
    assert 0.0 <= st["prepass_seconds"] <= st["first_submit_seconds"] <= st["seconds"]
    assert np.array_equal(res["best_score"], plain["best_score"])
    # hits: best first, ties to the lower index
    hs = res["best_score"][res["hits"]]
    assert np.all(np.diff(hs) >= 0)
    order = np.lexsort((np.arange(L), res["best_score"]))
    assert np.array_equal(res["hits"], order[:20])
    # the plain launch against the oracle, ligand by ligand
    grids = [O.Grid.of(p) for p in pockets]
    p = O.Params.of(s)
    ref = O.dock_batch(grids, p, library, per_orientation=True)
    for l in range(L):
        lig = library.ligand(l)
        a0, a1 = int(library.atom_offset[l]), int(library.atom_offset[l + 1])
        r = dict(best_k=int(ref["best_k"][l]), best_score=float(ref["best_score"][l]),
                 near_tie=ref["near_tie"][l])
        check_best_pose(O, grids[lig.pocket], p, lig, plain["best_score"][l], plain["desc"][l],
                        plain["coords"][a0:a1], ref=r)
    # the hit list against the oracle's: differences only at the cut, within tolerance
    ob = ref["best_score"]
    oracle_hits = set(np.lexsort((np.arange(L), ob))[:20].tolist())
    cut = float(np.sort(ob)[19])
    diff = oracle_hits ^ set(res["hits"].tolist())
    for l in diff:
        gap = abs(float(res["best_score"][l]) - ob[l])
        assert abs(ob[l] - cut) <= tol(cut) + gap, (l, ob[l], cut)
    log("hit list: %d of 20 shared with the oracle's" % (20 - len(diff) // 2))
