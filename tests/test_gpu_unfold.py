"""GPU unfolding of the input conformations (Sec. 3.1, first step) against the FP64 oracle,
alone and followed by docking.

A decision is a near tie when another turn's distance sum lies within the band
UNFOLD_PAIR_TOL * m * (n - m) of the kept one (a turn of m atoms changes only the m (n - m)
distances between turning and fixed atoms, each allowed 5e-5 A in FP32).  Where the oracle flags
no near tie among a ligand's decisions, the GPU must keep the same turns and reach the same
(re-centred) coordinates within 1e-4 A; otherwise every GPU decision is checked on its own
trajectory: replayed in FP64, the kept turn's sum is within the band of the largest, and the
replayed pose is the GPU's."""
import sys

import numpy as np
import pytest

import exs_synth as S
from parity import check_ligand

pytestmark = pytest.mark.gpu


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


class Lig:
    def __init__(self, xyz, types, bonds, rot, pocket=0):
        self.xyz = np.asarray(xyz, np.float32)
        self.types = np.asarray(types, np.uint8)
        self.bonds = np.asarray(bonds, np.int32)
        self.rot = np.asarray(rot, np.int32)
        self.pocket = pocket

    @property
    def n(self):
        return self.xyz.shape[0]


def centred(X):
    X = np.asarray(X, np.float64)
    return X - X.mean(axis=0)


def test_unfold_matches_oracle(B, oracle_lib):
    O = oracle_lib
    pocket = S.make_pocket("small")
    ligs = S.make_ligands("batched", 7, 32)
    ligs = [Lig(l.xyz, l.types % 4, l.bonds, l.rot) for l in ligs if l.n <= 128]
    batch = S.batch_from_ligands(ligs)
    R = int(batch.rot_offset[-1])
    A = int(batch.atom_offset[-1])
    pid = B.exs_load_pocket_grid(pocket.values, pocket.spacing, pocket.origin)
    try:
        bid = B.exs_upload_ligands(batch, pocket_ids=[pid])
        before = B.exs_get_ligand_coords(bid, A)
        assert B.exs_unfold_ligands(bid, 16, 0, n_rot=R) is None      # 0 passes: unchanged
        assert np.array_equal(B.exs_get_ligand_coords(bid, A), before)
        turns = B.exs_unfold_ligands(bid, 16, 2, n_rot=R)
        after = B.exs_get_ligand_coords(bid, A).astype(np.float64)
        B.exs_release_ligands(bid)
        one = B.exs_upload_ligands(batch.subset(range(1)), pocket_ids=[pid])
        with pytest.raises(B.ExsError) as ei:
            B.exs_unfold_ligands(one, 12, 1)                           # S must be 8, 16 or 32
        assert ei.value.code == B.EXS_EINVAL
        B.exs_release_ligands(one)
    finally:
        B.exs_unload_pocket(pid)
    exact = valid = 0
    for l, lig in enumerate(ligs):
        r0, r1 = int(batch.rot_offset[l]), int(batch.rot_offset[l + 1])
        a0, a1 = int(batch.atom_offset[l]), int(batch.atom_offset[l + 1])
        ref = O.unfold_ligand(lig, 16, 2)
        X = after[a0:a1]
        if ref["near_ties"] == 0:
            assert np.array_equal(turns[:, r0:r1], ref["turns"]), "ligand %d: turns differ" % l
            assert np.abs(X - centred(ref["xyz"])).max() < 1e-4, "ligand %d: coordinates" % l
            exact += 1
        else:
            validate_decisions(O, lig, 16, turns[:, r0:r1], X)
            valid += 1
        assert abs(X.mean(axis=0)).max() < 1e-4                        # re-centred
    log("unfold: %d exact, %d near-tie ligands validated decision by decision" % (exact, valid))
    assert 3 * exact >= 2 * len(ligs)


def validate_decisions(O, lig, S_, turns, X_gpu):
    """Replay the GPU's kept turns in FP64 from the input conformation: at every decision the
    kept turn's distance sum is within the near-tie band of the largest candidate's (so keeping
    it is a valid choice in FP32), and the replayed pose equals the GPU's."""
    u, v, moving = O.rot_topology(lig.n, lig.bonds, lig.rot)
    X = lig.xyz.astype(np.float64)
    for p in range(turns.shape[0]):
        for b in range(len(lig.rot)):
            cand = [O.distance_sum(X)] + [
                O.distance_sum(O.rotate_about_bond(X, u[b], v[b], moving[b], 2 * np.pi * s / S_))
                for s in range(1, S_)]
            t = int(turns[p, b])
            band = O.unfold_band(lig.n, int(moving[b].sum()))
            assert cand[t] >= max(cand) - band, (p, b, t, max(cand) - cand[t], band)
            if t:
                X = O.rotate_about_bond(X, u[b], v[b], moving[b], 2 * np.pi * t / S_)
    assert np.abs(X_gpu - centred(X)).max() < 1e-4


def test_unfold_then_dock_matches_oracle(B, oracle_lib):
    """Unfold on the GPU, then dock the unfolded batch; the oracle unfolds in FP64 and docks its
    own unfolded ligand (rounded to FP32), and the GPU results pass the usual parity checks."""
    O = oracle_lib
    pocket = S.make_pocket("small")
    g = O.Grid.of(pocket)
    s = S.SMALL.search
    base = S.make_ligands("small", 0, 12)
    batch = S.batch_from_ligands(base)
    pid = B.exs_load_pocket_grid(pocket.values, pocket.spacing, pocket.origin)
    try:
        bid = B.exs_upload_ligands(batch, pocket_ids=[pid])
        B.exs_unfold_ligands(bid, 16, 1)
        prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                              s.clash_cutoff, s.clash_penalty)
        job = B.exs_dock_batch(bid, prm)
        L, A = batch.n_ligands, int(batch.atom_offset[-1])
        best = B.exs_get_best_poses(job, L, A)
        orient = B.exs_get_orientation_results(job, L, s.n_orient)
        B.exs_release_job(job)
        B.exs_release_ligands(bid)
    finally:
        B.exs_unload_pocket(pid)
    stats, checked = {}, 0
    for l, lig in enumerate(base):
        ref = O.unfold_ligand(lig, 16, 1)
        if ref["near_ties"]:
            continue
        ul = Lig(ref["xyz"].astype(np.float32), lig.types, lig.bonds, lig.rot)
        a0, a1 = int(batch.atom_offset[l]), int(batch.atom_offset[l + 1])
        check_ligand(O, g, O.Params.of(s), ul, orient["score"][l], orient["desc"][l],
                     best["best_score"][l], best["desc"][l], best["coords"][a0:a1], stats=stats)
        checked += 1
    log("unfold + dock: %d ligands checked, stats %s" % (checked, stats))
    assert checked >= len(base) // 2
