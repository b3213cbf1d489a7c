"""The benchmark's algorithmic work counts (the roofline's numerator), checked on ligands whose
counts are worked out by hand, and the choice of the roofline's bound.  CPU only: the counts use
the library's host-side topology packing."""
import os
import sys

import numpy as np
import pytest

import exs_synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    import bench as bm
    return bm


@pytest.fixture(scope="module")
def B():
    from paper_2110_11644_amd import binding
    binding.lib()
    return binding


def chain(n, rot):
    xyz = np.array([[1.5 * i, 0.8 * (i % 2), 0.0] for i in range(n)], np.float32)
    bonds = np.array([[i, i + 1] for i in range(n - 1)], np.int32)
    return S.Ligand(xyz, np.zeros(n, np.uint8), bonds, np.asarray(rot, np.int32))


def test_counts_of_a_five_atom_chain(bench, B):
    """Chain 0-1-2-3-4, rotatable bond 1-2 (moving side {3, 4}), S=8, P=2, T=27.
    Lookups: 5 for the final score, and per pass 7 turns x 2 moving atoms plus 26 offsets x 5
    atoms: 5 + 2 (14 + 130) = 293.  Pairs more than three bonds apart: only (0, 4), which is also
    the bond's only (moving, static) pair: 1 + 2 x 1 = 3.  Turned positions: 2 x 7 x 2 = 28."""
    batch = S.batch_from_ligands([chain(5, [1])])
    search = S.SearchSettings(64, 8, 2, 27)
    L, Q, R = bench.algorithmic_counts(B, batch, search, 4)
    assert (L[0], Q[0], R[0]) == (293, 3, 28)


def test_counts_add_up_per_ligand(bench, B):
    """A rigid 3-atom ligand has no pair to test and no turn: L = 3 + 1 x 26 x 3 = 81 with one
    pass; a second ligand's counts are its own."""
    batch = S.batch_from_ligands([chain(3, []), chain(5, [1])])
    search = S.SearchSettings(64, 8, 1, 27)
    L, Q, R = bench.algorithmic_counts(B, batch, search, 4)
    assert (L[0], Q[0], R[0]) == (81, 0, 0)
    assert (L[1], Q[1], R[1]) == (5 + 14 + 130, 1 + 1, 14)


def test_roofline_bound_is_the_larger_fraction(bench, B):
    batch = S.batch_from_ligands([chain(5, [1])])
    search = S.SearchSettings(64, 8, 2, 27)
    roof = bench.roofline_of(B, batch, search, 4, kernel_ms=1e-3, storage=0, traffic=123.0)
    fr = {roof["bound"]: roof["frac"], roof["other"]["bound"]: roof["other"]["frac"]}
    assert set(fr) == {"texel-gather", "alu"}
    assert roof["frac"] >= roof["other"]["frac"]
    assert roof["traffic"] == 123.0
    # 8 corners x 4 bytes x 64 orientations x 293 lookups in 1 microsecond
    assert fr["texel-gather"] == pytest.approx(8 * 4 * 64 * 293 / 1e-6 / 1e9 / 8000.0, rel=1e-3)
    mem = roof if roof["bound"] == "texel-gather" else roof["other"]
    assert mem["dram"]["achieved"] == pytest.approx(123.0 / 1e-6 / 1e9)
    # every turn tested: 64 x (30 x 293 + 7 x (1 + 7 x 2) + 15 x 28) lane-ops in 1 microsecond
    alu = roof if roof["bound"] == "alu" else roof["other"]
    assert alu["frac_if_every_turn_tested"] == pytest.approx(
        64 * (30 * 293 + 7 * (1 + 7 * 2) + 15 * 28) / 1e-6 / 1e12 / bench.VALU_PEAK_TOPS, abs=1e-4)


def test_method_step_counts_of_a_five_atom_chain(bench, B):
    """Chain 0-1-2-3-4, rotatable bond 1-2 (moving side {3, 4}, m = 2), S=8, K=64, 2 unfolding
    passes, 3 clusters, 30 ranked poses kept.  Unfolding: 2 x 8 x 2 x (9 x 3 + 12) = 1,248.
    Ranking: 64^2 + 2 x 64 x 3 x 15 = 9,856.  Rescoring: c0 = 1 pair (0, 4), one bond, so
    30 x (30 x 5 + 12 x 1 + 40 x 1 + 20 x (5 + 2)) = 30 x 342 = 10,260."""
    batch = S.batch_from_ligands([chain(5, [1])])
    search = S.SearchSettings(64, 8, 2, 27)
    w = bench.method_work(B, batch, search, 4, np.array([3]), 30, 2)
    assert w == {"unfold": 1248, "rank": 9856, "rescore2": 10260}
    r = bench.step_roofline(w["rank"], 1e-3)   # 9,856 lane-ops in 1 microsecond
    assert r["bound"] == "alu" and r["frac"] == pytest.approx(9856 / 1e-6 / 1e12 / bench.VALU_PEAK_TOPS, abs=1e-4)
