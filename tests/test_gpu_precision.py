"""Mixed precision at the full search settings (256 orientations, 32 torsion steps, 2 passes,
27 rigid offsets), through the C ABI, against the FP64 oracle.

16-bit texels (BF16 and FP16, round to nearest even from the FP32 master) with FP32
interpolation and accumulation: every orientation of every ligand passes the FP32 acceptance
(tests/parity.py) against the oracle searching the same RNE-rounded grid.  The top-8 poses of
each ligand are rescored in FP64 on the GPU from the FP32 master grid: each rescored score equals
the oracle's FP64 score of the same descriptor on the master (rigid offsets tau != 0 included),
the top-8 list is the 8 lowest FP32 scores, and the final best is the FP64 argmin of the list,
with its FP64 coordinates.
"""
import sys

import numpy as np
import pytest

import exs_synth as S
from parity import check_ligand, gpu_desc_to_theta_tau

pytestmark = pytest.mark.gpu

FULL = S.SearchSettings(256, 32, 2, 27)
TOP_K = 8
ROUNDERS = {1: S.to_bf16_rne, 2: S.to_f16_rne}


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


def dock(B, pockets, batch, search, storage, top_k, flags=0):
    pids = [B.exs_load_pocket_grid(p.values, p.spacing, p.origin, storage) for p in pockets]
    try:
        bid = B.exs_upload_ligands(batch, pocket_ids=pids)
        prm = B.search_params(search.n_orient, search.torsion_steps, search.passes,
                              search.n_offsets, search.offset_step, search.clash_cutoff,
                              search.clash_penalty, top_k=top_k, flags=flags)
        job = B.exs_dock_batch(bid, prm)
        L, A = batch.n_ligands, int(batch.atom_offset[-1])
        best = B.exs_get_best_poses(job, L, A, top_k=top_k)
        orient = B.exs_get_orientation_results(job, L, search.n_orient)
        B.exs_release_job(job)
        B.exs_release_ligands(bid)
    finally:
        for pid in pids:
            B.exs_unload_pocket(pid)
    return dict(best_score=best["best_score"], best=best["desc"], coords=best["coords"],
                topk=best["topk"].reshape(batch.n_ligands, top_k), score=orient["score"],
                desc=orient["desc"])


def check_topk_fp64(O, g_master, prm, lig, out, l, a0, a1):
    """FP64 rescoring of the top_k list of ligand l; returns how many of its descriptors carry
    a nonzero rigid offset."""
    top = out["topk"][l]
    sc = out["score"][l]
    order = sorted(range(len(sc)), key=lambda k: (sc[k], k))[:TOP_K]
    assert [int(d["orient"]) for d in top] == order
    e64, moved = [], 0
    for d in top:
        th, ta = gpu_desc_to_theta_tau(d, len(lig.rot))
        e, _, amb = O.rescore_desc(g_master, prm, lig, int(d["orient"]), th, ta)[:3]
        assert abs(float(d["score_fp64"]) - e) <= 1e-9 * max(1.0, abs(e)) + prm.clash_penalty * amb, (
            "ligand %d, orientation %d: fp64 %.12g vs oracle %.12g" % (l, d["orient"], d["score_fp64"], e))
        assert float(d["score"]) == float(sc[int(d["orient"])])
        e64.append(float(d["score_fp64"]))
        moved += int(np.any(ta != 0))
    j = int(np.argmin(e64))
    best = out["best"][l]
    assert int(best["orient"]) == int(top[j]["orient"])
    assert float(best["score_fp64"]) == e64[j]
    assert float(out["best_score"][l]) == np.float32(e64[j])
    th, ta = gpu_desc_to_theta_tau(top[j], len(lig.rot))
    X = O.pose_from_desc(g_master, prm, lig, int(top[j]["orient"]), th, ta)
    assert np.max(np.abs(out["coords"][a0:a1] - X)) < 1e-5
    return moved


def check_run(O, grids16, grids32, prm, batch, out, idx):
    stats, moved = {}, 0
    for l in idx:
        lig = batch.ligand(l)
        a0, a1 = int(batch.atom_offset[l]), int(batch.atom_offset[l + 1])
        # the search against the oracle on the rounded grid (best = FP32 argmin, topk[0])
        t0 = out["topk"][l][0]
        check_ligand(O, grids16[lig.pocket], prm, lig, out["score"][l], out["desc"][l],
                     t0["score"], t0, None, stats=stats)
        moved += check_topk_fp64(O, grids32[lig.pocket], prm, lig, out, l, a0, a1)
    return stats, moved


@pytest.mark.parametrize("storage", [1, 2], ids=["bf16", "f16"])
def test_16bit_full_search_small_pocket(B, oracle_lib, storage):
    """8 ligands of the oracle-sized workload (24 atoms, 4 rotatable bonds) in its 48^3 x 4
    pocket, at the full search settings, one launch per pocket."""
    O = oracle_lib
    p = S.make_pocket("small")
    batch = S.make_ligand_batch("small", 0, 8)
    log("16-bit full search, small pocket, storage %d" % storage)
    out = dock(B, [p], batch, FULL, storage, TOP_K)
    g16 = O.Grid(ROUNDERS[storage](p.values), p.spacing, p.origin)
    stats, moved = check_run(O, [g16], [O.Grid.of(p)], O.Params.of(FULL), batch, out,
                             range(batch.n_ligands))
    log("stats", stats, "top-8 descriptors with tau != 0:", moved)
    assert moved > 0, "no rescored pose carried a rigid offset"
    assert stats["near_tie"] < 0.6 * stats["orientations"]


@pytest.mark.parametrize("storage", [1, 2], ids=["bf16", "f16"])
def test_16bit_full_search_batched_sample(B, oracle_lib, storage):
    """3 seeded ligands of the batched workload, each in its own batched pocket (edges up to
    128), in one persistent launch over those pockets, as the precision benchmark runs."""
    O = oracle_lib
    wl = S.BATCHED
    rng = np.random.default_rng(20211013)
    picks = sorted(rng.choice(2000, size=3, replace=False).tolist())
    full = S.make_ligand_batch(wl, 0, 2000)
    ligs = [full.ligand(l) for l in picks]
    used = sorted(set(l.pocket for l in ligs))
    pockets = [S.make_pocket(wl, i) for i in used]
    for l in ligs:
        l.pocket = used.index(l.pocket)
    batch = S.batch_from_ligands(ligs)
    log("16-bit full search, batched ligands %s (n %s, bonds %s), pockets %s, storage %d" % (
        picks, [l.n for l in ligs], [len(l.rot) for l in ligs], used, storage))
    out = dock(B, pockets, batch, FULL, storage, TOP_K, flags=B.EXS_FLAG_PERSISTENT)
    g16 = [O.Grid(ROUNDERS[storage](p.values), p.spacing, p.origin) for p in pockets]
    g32 = [O.Grid.of(p) for p in pockets]
    stats, moved = check_run(O, g16, g32, O.Params.of(FULL), batch, out, range(batch.n_ligands))
    log("stats", stats, "top-8 descriptors with tau != 0:", moved)
    assert moved > 0
