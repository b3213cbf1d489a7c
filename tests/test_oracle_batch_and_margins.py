"""Pins of the oracle's batch wrapper and of its near-tie bookkeeping (CPU).

* The multi-pocket CSR wrapper (OpenMP over ligands) must give, ligand for ligand, exactly what
  the single-ligand search gives with the ligand's own pocket: best orientation and score, and
  every orientation's score, near-tie flag, torsions and offsets.  The batch is uneven (1 to 20
  atoms, 0 to 4 rotatable bonds, a ligand without rotatable bonds between others) over three
  pockets of different edges and values, so a slip in the CSR slices, the per-ligand output
  offsets or the pocket index gives a different answer.
* The near-tie flag of a decision (Sec. 3.1: the greedy search keeps the best candidate; the
  flag marks decisions another precision could take differently) is pinned by constructed
  candidate sets: a gap below the tolerance flags, above it does not, the tolerance is relative
  to max(|e|, 1), and every ambiguous clash pair widens the gap allowance by one penalty.  End
  to end, a single clash pair whose distance sits 5e-5 A from the cutoff flags the decision, one
  2e-4 A away does not.
"""
import numpy as np
import pytest

import exs_synth as S

WL = S.Workload("pin-batch", 93, 14, 3, (20, 24, 28), 0.5, 4, ("uniform", 1, 20),
                ("uniform", 0, 4), S.SearchSettings(8, 8, 2, 27))


class Lig:
    def __init__(self, xyz, types, bonds, rot=(), pocket=0):
        self.xyz = np.asarray(xyz, np.float32)
        self.types = np.asarray(types, np.uint8)
        self.bonds = np.asarray(bonds, np.int32).reshape(-1, 2)
        self.rot = np.asarray(rot, np.int32)
        self.pocket = pocket

    @property
    def n(self):
        return self.xyz.shape[0]


@pytest.fixture(scope="module")
def three_pockets():
    pockets = [S.make_pocket(WL, i) for i in range(3)]
    edges = [p.n for p in pockets]
    if len(set(edges)) < 2:          # the pin needs pockets that differ in shape as well
        pockets[1] = S.make_pocket(S.Workload("pin-batch-b", 94, 0, 1, (20,), 0.5, 4, ("fixed", 2),
                                              ("fixed", 0), WL.search), 0)
    return pockets


def _uneven_batch():
    ligs = S.make_ligands(WL, 0, WL.n_ligands)
    pocket_of = [2, 0, 1, 1, 2, 0, 0, 2, 1, 0, 2, 1, 0, 2]
    for l, p in zip(ligs, pocket_of):
        l.pocket = p
    # a ligand without rotatable bonds, and a one-atom ligand, between the others
    ligs[4] = S.Ligand(ligs[4].xyz, ligs[4].types, ligs[4].bonds, np.zeros(0, np.int32), 2)
    ligs[7] = S.Ligand(np.array([[0.4, -0.3, 0.2]], np.float32), np.array([3], np.uint8),
                       np.zeros((0, 2), np.int32), np.zeros(0, np.int32), 2)
    return ligs


@pytest.mark.parametrize("threads", [1, 4])
def test_dock_batch_equals_single_ligand_search(oracle_lib, three_pockets, threads):
    O = oracle_lib
    grids = [O.Grid.of(p) for p in three_pockets]
    prm = O.Params.of(WL.search)
    ligs = _uneven_batch()
    batch = S.batch_from_ligands(ligs)
    nrot = np.diff(batch.rot_offset)
    assert nrot.min() == 0 and nrot.max() >= 2 and len(set(np.diff(batch.atom_offset))) > 4
    r = O.dock_batch(grids, prm, batch, threads=threads, per_orientation=True)
    K = prm.n_orient
    for l, lig in enumerate(ligs):
        ref = O.dock_ligand(grids[lig.pocket], prm, lig)
        assert r["best_k"][l] == ref["best_k"], l
        assert r["best_score"][l] == ref["best_score"], l
        assert np.array_equal(r["score"][l], ref["score"]), l
        assert np.array_equal(r["near_tie"][l], ref["near_tie"]), l
        assert np.array_equal(r["tau"][l], ref["tau"]), l
        r0, nr = int(batch.rot_offset[l]), int(nrot[l])
        th = r["theta"][r0 * K:r0 * K + K * nr].reshape(K, nr)
        assert np.array_equal(th, ref["theta"]), l
    # the pocket index matters: the same ligands against another pocket score differently
    other = S.batch_from_ligands([S.Ligand(x.xyz, x.types, x.bonds, x.rot, (x.pocket + 1) % 3)
                                  for x in ligs])
    r2 = O.dock_batch(grids, prm, other, threads=threads)
    assert not np.array_equal(r2["best_score"], r["best_score"])


def test_dock_batch_rejects_an_unknown_pocket(oracle_lib, three_pockets):
    O = oracle_lib
    grids = [O.Grid.of(p) for p in three_pockets]
    ligs = _uneven_batch()[:3]
    ligs[1].pocket = 3
    with pytest.raises(ValueError):
        O.dock_batch(grids, O.Params.of(WL.search), S.batch_from_ligands(ligs), threads=2)


def tol(e):
    return 1e-4 * max(abs(e), 1.0)


@pytest.mark.parametrize("e0", [10.0, -200.0, 0.5, 0.0])
def test_gap_below_the_tolerance_flags(oracle_lib, e0):
    O = oracle_lib
    t = tol(e0)
    assert O.decision_margin([e0, e0 + 0.5 * t], 0)[0]
    assert not O.decision_margin([e0, e0 + 2.0 * t], 0)[0]
    # the tolerance is relative to the chosen candidate's score, with max(|e|, 1)
    assert O.decision_margin([e0 + 3 * t, e0, e0 + 0.9 * t], 1)[0]
    assert not O.decision_margin([e0 + 3 * t, e0, e0 + 1.1 * t], 1)[0]
    near, gap = O.decision_margin([e0 + 3 * t, e0, e0 + 1.1 * t], 1)
    assert gap == pytest.approx(1.1 * t, rel=1e-6)


def test_tolerance_floor_is_one_not_the_score(oracle_lib):
    O = oracle_lib
    # |e| = 0.5 < 1: the tolerance is 1e-4, not 0.5e-4
    assert O.decision_margin([0.5, 0.5 + 0.8e-4], 0)[0]
    assert not O.decision_margin([0.5, 0.5 + 1.2e-4], 0)[0]


def test_exact_tie_and_single_candidate(oracle_lib):
    O = oracle_lib
    assert O.decision_margin([3.0, 3.0], 0)[0]
    near, gap = O.decision_margin([3.0], 0)
    assert not near and gap == float("inf")


@pytest.mark.parametrize("penalty", [1.0, 2.5])
def test_ambiguous_pairs_widen_the_gap_by_one_penalty_each(oracle_lib, penalty):
    O = oracle_lib
    e0 = 20.0
    t = tol(e0)
    # one ambiguous pair on one side: allowance = penalty (counted once)
    assert not O.decision_margin([e0, e0 + penalty + 2 * t], 0, [1, 0], clash_penalty=penalty)[0]
    assert O.decision_margin([e0, e0 + penalty + 0.5 * t], 0, [1, 0], clash_penalty=penalty)[0]
    assert not O.decision_margin([e0, e0 + penalty + 2 * t], 0, [0, 1], clash_penalty=penalty)[0]
    # one on each side: allowance = 2 penalties
    assert O.decision_margin([e0, e0 + 1.5 * penalty], 0, [1, 1], clash_penalty=penalty)[0]
    assert not O.decision_margin([e0, e0 + 2 * penalty + 2 * t], 0, [1, 1],
                                 clash_penalty=penalty)[0]
    near, gap = O.decision_margin([e0, e0 + 5.0], 0, [2, 1], clash_penalty=penalty)
    assert gap == pytest.approx(5.0 - 3 * penalty, rel=1e-12)


def _pair_near_cutoff_search(O, delta):
    """Five-atom chain (only the pair 0-4 is at bond distance >= 4) whose atoms 0 and 4 are
    2.0 + delta A apart, K = 1 orientation, no rotatable bond, one pass of the 27 rigid offsets
    on the shallow ramp 0.01 (x + 3y + 9z): the 27 offsets score 0.025 (a + 3b + 9c) apart,
    all different, far above the tolerance and far below one clash penalty.  Rigid offsets keep
    the pair distance, so the pair is ambiguous in every candidate or in none."""
    n, h = 40, 0.5
    ax = np.arange(n, dtype=np.float64) * h - h * (n - 1) / 2.0
    ramp = 0.01 * (ax[None, None, :] + 3.0 * ax[None, :, None] + 9.0 * ax[:, None, None])
    vals = ramp.astype(np.float32)[None]
    g = O.Grid(np.ascontiguousarray(vals), h, [-h * (n - 1) / 2.0] * 3)
    xyz = [[0.0, 0.0, 0.0], [0.7, 1.3, 0.0], [1.5, 2.4, 0.3], [2.2, 1.2, -0.2],
           [2.0 + delta, 0.0, 0.0]]
    lig = Lig(xyz, [0] * 5, [[0, 1], [1, 2], [2, 3], [3, 4]])
    X = lig.xyz.astype(np.float64)
    assert abs(np.linalg.norm(X[0] - X[4]) - (2.0 + delta)) < 1e-6
    return O.dock_ligand(g, O.Params(1, 8, 1, 27), lig)


@pytest.mark.parametrize("delta,flag", [(5e-5, True), (-5e-5, True), (2e-4, False), (-2e-4, False)])
def test_clash_pair_within_the_band_flags_the_decision(oracle_lib, delta, flag):
    O = oracle_lib
    r = _pair_near_cutoff_search(O, delta)
    assert bool(r["ambiguous"][0]) == flag
    assert bool(r["near_tie"][0]) == flag
    assert r["clashes"][0] == (1 if delta < 0 else 0)
    assert r["tau"][0].tolist() == [-1, -1, -1]     # the lowest ramp value wins
