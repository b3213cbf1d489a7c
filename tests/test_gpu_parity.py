"""GPU parity of the HIP docking path against the FP64 oracle (through the C ABI).

Acceptance per ligand is in tests/parity.py (per-pose score within 1e-4
relative, trajectories equal except on oracle-flagged near ties, best pose
within tolerance with ties accepted, best-pose RMSD <= 0.01 A).
"""
import math
import sys

import numpy as np
import pytest

import exs_synth as S
from parity import check_ligand, tol

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
    def __init__(self, xyz, types, bonds, rot=(), pocket=0):
        self.xyz = np.asarray(xyz, np.float32)
        self.types = np.asarray(types, np.uint8)
        self.bonds = np.asarray(bonds, np.int32).reshape(-1, 2)
        self.rot = np.asarray(rot, np.int32)
        self.pocket = pocket

    @property
    def n(self):
        return self.xyz.shape[0]


def run(B, pockets, batch, search, storage=0, top_k=0, ppl=0, lpw=0, flags=0, orient=True):
    """Load pockets, upload, dock, fetch, release.  Returns numpy results:
    best_score [L], best [L] (descriptors), coords [A,3], topk, score [L,K], desc [L,K], ms."""
    pids = [B.exs_load_pocket_grid(p.values, p.spacing, p.origin, storage) for p in pockets]
    bid = B.exs_upload_ligands(batch, pocket_ids=pids)
    prm = B.search_params(search.n_orient, search.torsion_steps, search.passes, search.n_offsets,
                          search.offset_step, search.clash_cutoff, search.clash_penalty,
                          top_k=top_k, poses_per_lane=ppl, ligands_per_wg=lpw, flags=flags)
    job = B.exs_dock_batch(bid, prm)
    L, A = batch.n_ligands, int(batch.atom_offset[-1])
    best = B.exs_get_best_poses(job, L, A, top_k=top_k)
    out = dict(best_score=best["best_score"], best=best["desc"], coords=best["coords"],
               topk=best["topk"])
    if orient:
        out.update(B.exs_get_orientation_results(job, L, search.n_orient))
    out["ms"] = B.exs_job_elapsed_ms(job)
    B.exs_release_job(job)
    B.exs_release_ligands(bid)
    for pid in pids:
        B.exs_unload_pocket(pid)
    return out


def check_all(O, grids, prm, batch, out, idx=None, refs=None):
    stats = {}
    idx = list(range(batch.n_ligands)) if idx is None else list(idx)
    for j, l in enumerate(idx):
        lig = batch.ligand(l)
        a0, a1 = int(batch.atom_offset[l]), int(batch.atom_offset[l + 1])
        check_ligand(O, grids[lig.pocket], prm, lig, out["score"][l], out["desc"][l],
                     out["best_score"][l], out["best"][l], out["coords"][a0:a1],
                     ref=None if refs is None else refs[j], stats=stats)
    return stats


@pytest.fixture(scope="module")
def small(oracle_lib):
    p = S.make_pocket("small")
    return p, oracle_lib.Grid.of(p), S.make_ligand_batch("small")


def test_small_workload_full_parity(B, oracle_lib, small):
    O = oracle_lib
    p, g, batch = small
    s = S.SMALL.search
    log("small workload: 64 ligands x 64 orientations, FP32")
    out = run(B, [p], batch, s)
    stats = check_all(O, [g], O.Params.of(s), batch, out)
    log("small workload stats:", stats, "ms", out["ms"])
    assert stats["near_tie"] < 0.25 * stats["orientations"]


def test_tile_configs_and_persistent_are_bitwise_identical(B, small):
    p, g, batch = small
    s = S.SMALL.search
    ref = None
    for ppl, lpw, flags in [(1, 1, 0), (2, 1, 0), (1, 4, 0), (1, 8, 0),
                            (1, 2, B.EXS_FLAG_PERSISTENT), (2, 4, B.EXS_FLAG_PERSISTENT)]:
        log("tile config ppl=%d lpw=%d flags=%d" % (ppl, lpw, flags))
        out = run(B, [p], batch, s, ppl=ppl, lpw=lpw, flags=flags)
        key = (out["score"], out["desc"]["theta"], out["desc"]["tau"], out["coords"],
               out["best_score"])
        if ref is None:
            ref = key
        else:
            for a, b in zip(ref, key):
                assert np.array_equal(a, b)


def test_every_tile_of_the_tuner_is_bitwise_identical(B, small):
    """All twelve (poses per lane, ligands per workgroup) tiles at 256 orientations and 32
    torsion steps, one launch per pocket and persistent: the tiles with more orientation chunks
    than a workgroup has waves (ligands per workgroup 4 and 8 at one or two poses per lane), and
    four poses per lane, whose LDS difference arrays cap the workgroup's waves, give the results
    of (1, 1) bit for bit."""
    p, g, batch = small
    s = S.SearchSettings(256, 32, 1, 27)
    sub = batch.subset(range(20))
    ref = None
    for ppl in (1, 2, 4):
        for lpw in (1, 2, 4, 8):
            for flags in (0, B.EXS_FLAG_PERSISTENT):
                log("tile ppl=%d lpw=%d flags=%d" % (ppl, lpw, flags))
                out = run(B, [p], sub, s, ppl=ppl, lpw=lpw, flags=flags)
                key = (out["score"], out["desc"]["theta"], out["desc"]["tau"], out["coords"],
                       out["best_score"])
                if ref is None:
                    ref = key
                else:
                    for a, b in zip(ref, key):
                        assert np.array_equal(a, b), (ppl, lpw, flags)


def test_orientation_count_not_a_multiple_of_64(B, oracle_lib, small):
    O = oracle_lib
    p, g, batch = small
    s = S.SearchSettings(100, 16, 1, 27)
    sub = batch.subset(range(6))
    log("K=100, T=27, 6 ligands")
    out = run(B, [p], sub, s, ppl=2)
    check_all(O, [g], O.Params.of(s), sub, out)


def test_brute_force_tiny_ligands_on_gpu(B, oracle_lib, small):
    """3-atom ligands (one pass, 27 offsets: exhaustive over K x 27 poses) and 4-atom chains
    with one rotatable bond (exhaustive over K x S): the GPU finds the oracle's optimum."""
    O = oracle_lib
    p, g, _ = small
    rng = np.random.default_rng(11)
    half = math.radians(109.5) / 2
    tri = np.array([[0, 0, 0], [1.5, 0, 0], [1.5 * math.cos(2 * half), 1.5 * math.sin(2 * half), 0]])
    ligs = [Lig(tri + rng.normal(scale=0.05, size=(3, 3)), rng.integers(0, 4, 3), [[0, 1], [0, 2]])
            for _ in range(8)]
    zig = np.array([[k * 1.5 * math.sin(half), (k % 2) * 1.5 * math.cos(half), 0.0] for k in range(4)])
    chains = [Lig(zig + rng.normal(scale=0.02, size=(4, 3)), rng.integers(0, 4, 4),
                  [[0, 1], [1, 2], [2, 3]], [1]) for _ in range(8)]
    for name, group, s in (("3-atom", ligs, S.SearchSettings(16, 8, 1, 27)),
                           ("4-atom chain", chains, S.SearchSettings(16, 16, 1, 1))):
        log("brute force:", name)
        batch = S.batch_from_ligands(group)
        out = run(B, [p], batch, s)
        prm = O.Params.of(s)
        for l, lig in enumerate(group):
            r = O.dock_ligand(g, prm, lig)
            assert abs(float(out["best_score"][l]) - r["best_score"]) <= tol(r["best_score"])
            k = int(out["best"][l]["orient"])
            if k != r["best_k"]:
                assert r["near_tie"][k] or r["near_tie"][r["best_k"]]
            elif not r["near_tie"][k]:
                assert out["best"][l]["tau"].tolist() == r["tau"][k].tolist()
                assert out["best"][l]["theta"][:len(lig.rot)].tolist() == r["theta"][k].tolist()


def test_degenerate_ligands_and_one_orientation(B, oracle_lib, small):
    """Single-atom and two-atom ligands (no pairs to clash, no rotatable bond), a ligand whose
    rotatable bond turns one atom, a rotatable bond that turns no atom (its far end is
    terminal), and K = 1 (one restart): full acceptance against the oracle."""
    O = oracle_lib
    p, g, _ = small
    ligs = [Lig([[0.3, -0.2, 0.1]], [2], np.zeros((0, 2), np.int32)),
            Lig([[0, 0, 0], [1.5, 0, 0]], [0, 3], [[0, 1]]),
            Lig([[0, 0, 0], [1.5, 0, 0], [2.0, 1.4, 0], [3.5, 1.4, 0.2]], [1, 2, 3, 0],
                [[0, 1], [1, 2], [2, 3]], [1]),
            Lig([[0, 0, 0], [1.5, 0, 0], [2.0, 1.4, 0]], [3, 1, 2], [[0, 1], [1, 2]], [1])]
    batch = S.batch_from_ligands(ligs)
    for s in (S.SearchSettings(8, 8, 1, 27), S.SearchSettings(1, 16, 2, 27), S.SearchSettings(64, 32, 1, 1)):
        log("degenerate ligands, K=%d S=%d P=%d T=%d" % (s.n_orient, s.torsion_steps, s.passes, s.n_offsets))
        out = run(B, [p], batch, s)
        check_all(O, [g], O.Params.of(s), batch, out)


def test_largest_ligands_use_all_mask_words(B, oracle_lib, small):
    """n = 128 atoms and 32 rotatable bonds (the limits): every 32-bit word of the masks."""
    O = oracle_lib
    p, g, _ = small
    wl = S.Workload("limits", 90, 2, 1, (48,), 0.5, 4, ("fixed", 128), ("fixed", 32),
                    S.SearchSettings(8, 8, 1, 27))
    ligs = S.make_ligands(wl, 0, 2)
    big = [l for l in S.make_ligands("batched", 0, 400) if l.n >= 80][:1]
    ligs += [S.Ligand(b.xyz, b.types % 4, b.bonds, b.rot) for b in big]
    batch = S.batch_from_ligands(ligs)
    log("limits: n=%s B=%s" % ([l.n for l in ligs], [len(l.rot) for l in ligs]))
    out = run(B, [p], batch, wl.search)
    check_all(O, [g], O.Params.of(wl.search), batch, out)


def test_multi_pocket_persistent_and_per_pocket_agree(B, oracle_lib):
    """Uneven ligands over three pockets of different edges: one persistent launch equals the
    per-pocket launches bitwise, and a sample matches the oracle."""
    O = oracle_lib
    wl = S.Workload("mixed", 91, 36, 3, (24, 32, 40), 0.375, 8, ("lognormal", 35.0, 0.4, 10, 90),
                    ("uniform", 0, 15), S.SearchSettings(64, 8, 1, 27))
    pockets = [S.make_pocket(wl, i) for i in range(3)]
    grids = [O.Grid.of(pk) for pk in pockets]
    batch = S.make_ligand_batch(wl, 0, 36)
    log("mixed pockets: edges", [pk.n for pk in pockets])
    a = run(B, pockets, batch, wl.search)
    b = run(B, pockets, batch, wl.search, flags=B.EXS_FLAG_PERSISTENT, lpw=2)
    for key in ("score", "best_score", "coords"):
        assert np.array_equal(a[key], b[key])
    assert np.array_equal(a["desc"]["theta"], b["desc"]["theta"])
    stats = check_all(O, grids, O.Params.of(wl.search), batch, a, idx=range(0, 36, 4))
    log("mixed stats", stats)


def test_pocket_major_persistent_launch_equals_per_pocket(B):
    """A persistent launch large enough for the pocket-major work queues (each pocket holds
    more ligands than the device has in flight: 3,072 one-wave ligands at 64 orientations)
    equals the per-pocket launches bitwise, at one and two ligands per workgroup."""
    wl = S.Workload("pocketmajor", 92, 7000, 2, (32, 40), 0.375, 8, ("uniform", 10, 24),
                    ("uniform", 0, 4), S.SearchSettings(64, 8, 1, 27))
    pockets = [S.make_pocket(wl, i) for i in range(2)]
    batch = S.make_ligand_batch(wl, 0, wl.n_ligands)
    per_pocket = np.bincount([batch.ligand(l).pocket for l in range(batch.n_ligands)], minlength=2)
    log("pocket-major: ligands per pocket", per_pocket.tolist())
    assert per_pocket.min() >= 3072
    a = run(B, pockets, batch, wl.search)
    for lpw in (1, 2):
        b = run(B, pockets, batch, wl.search, flags=B.EXS_FLAG_PERSISTENT, lpw=lpw)
        for key in ("score", "best_score", "coords"):
            assert np.array_equal(a[key], b[key]), (lpw, key)
        assert np.array_equal(a["desc"]["theta"], b["desc"]["theta"])
        assert np.array_equal(a["best"]["orient"], b["best"]["orient"])


@pytest.mark.parametrize("storage", [0, 1, 2], ids=["f32", "bf16", "f16"])
def test_odd_unequal_grid_edges(B, oracle_lib, small, storage):
    """A grid with odd, unequal edges (x 45, y 38, z 41 texels) cut from the small pocket, so
    that the cell blocks at the odd edges are padding and many atoms fall outside the grid and
    are clamped to its faces: each texel storage matches the oracle on the same grid (for
    16-bit storage the oracle reads the grid rounded by numpy)."""
    import types
    O = oracle_lib
    p, _, batch = small
    vals = np.ascontiguousarray(p.values[:, :41, :38, :45])
    cut = types.SimpleNamespace(values=vals, spacing=p.spacing, origin=p.origin)
    ref_vals = vals if storage == 0 else (S.to_bf16_rne if storage == 1 else S.to_f16_rne)(vals)
    g = O.Grid(ref_vals, p.spacing, p.origin)
    s = S.SMALL.search
    sub = batch.subset(range(12))
    log("odd grid 45x38x41, storage %d" % storage)
    out = run(B, [cut], sub, s, storage=storage)
    stats = check_all(O, [g], O.Params.of(s), sub, out)
    log("odd grid stats", stats)


def test_invalid_requests_fail_alone(B, small):
    p, g, batch = small
    pid = B.exs_load_pocket_grid(p.values, p.spacing, p.origin)
    try:
        bad = batch.subset(range(3))
        bad.type[5] = 4                                 # channel out of range
        with pytest.raises(B.ExsError) as ei:
            B.exs_upload_ligands(bad, pocket_ids=[pid])
        assert ei.value.code == B.EXS_EINVAL
        with pytest.raises(B.ExsError) as ei:
            B.exs_upload_ligands(batch.subset(range(3)), pocket_ids=[pid + 1000])
        assert ei.value.code == B.EXS_EINVAL
        bid = B.exs_upload_ligands(batch.subset(range(3)), pocket_ids=[pid])
        for kw in (dict(n_orient=0), dict(torsion_steps=12), dict(n_offsets=9), dict(top_k=64)):
            d = dict(n_orient=8, torsion_steps=8, passes=1, n_offsets=1)
            d.update(kw)
            with pytest.raises(B.ExsError) as ei:
                B.exs_dock_batch(bid, B.search_params(**d))
            assert ei.value.code == B.EXS_EINVAL
        job = B.exs_dock_batch(bid, B.search_params(8, 8, 1, 1))
        out = B.exs_get_best_poses(job, 3, int(batch.atom_offset[3]))
        assert np.all(np.isfinite(out["best_score"]))
        with pytest.raises(B.ExsError):
            B.exs_release_ligands(bid)                  # job still holds it
        B.exs_release_job(job)
        B.exs_release_ligands(bid)
        empty = S.batch_from_ligands([])
        bid = B.exs_upload_ligands(empty, pocket_ids=[pid])
        job = B.exs_dock_batch(bid, B.search_params(8, 8, 1, 1))
        B.exs_get_best_poses(job, 0, 0)
        B.exs_release_job(job)
        B.exs_release_ligands(bid)
    finally:
        B.exs_unload_pocket(pid)


@pytest.mark.parametrize("storage,rounder", [(1, S.to_bf16_rne), (2, S.to_f16_rne)],
                         ids=["bf16", "f16"])
def test_16bit_texels_match_oracle_on_rounded_grid(B, oracle_lib, small, storage, rounder):
    """BF16/FP16 storage with FP32 interpolation equals the FP32 path on the RNE-rounded grid:
    the oracle, fed that rounded grid, is the reference (rounding done by numpy)."""
    O = oracle_lib
    p, _, batch = small
    s = S.SMALL.search
    sub = batch.subset(range(16))
    log("16-bit storage %d" % storage)
    out = run(B, [p], sub, s, storage=storage)
    g16 = O.Grid(rounder(p.values), p.spacing, p.origin)
    stats = check_all(O, [g16], O.Params.of(s), sub, out)
    log("16-bit stats", stats)


def check_topk(O, g, s, sub, out, tk):
    """top_k descriptors are the K best FP32 poses, each FP64 score equals the oracle's FP64
    score of the same descriptor, and the final best is their FP64 argmin."""
    prm = O.Params.of(s)
    for l in range(sub.n_ligands):
        lig = sub.ligand(l)
        top = out["topk"][l]
        sc = out["score"][l]
        order = sorted(range(s.n_orient), key=lambda k: (sc[k], k))[:tk]
        assert [int(d["orient"]) for d in top] == order
        e64 = []
        for d in top:
            e, _, amb = O.rescore_desc(g, prm, lig, int(d["orient"]), d["theta"][:len(lig.rot)],
                                       d["tau"])[:3]
            assert abs(float(d["score_fp64"]) - e) <= 1e-9 * max(1.0, abs(e)) + prm.clash_penalty * amb
            assert float(d["score"]) == float(sc[int(d["orient"])])
            e64.append(float(d["score_fp64"]))
        j = int(np.argmin(e64))
        assert int(out["best"][l]["orient"]) == int(top[j]["orient"])
        assert float(out["best"][l]["score_fp64"]) == e64[j]
        assert float(out["best_score"][l]) == np.float32(e64[j])
        a0, a1 = int(sub.atom_offset[l]), int(sub.atom_offset[l + 1])
        X = O.pose_from_desc(g, prm, lig, int(top[j]["orient"]), top[j]["theta"][:len(lig.rot)],
                             top[j]["tau"])
        assert np.max(np.abs(out["coords"][a0:a1] - X)) < 1e-5


def test_fp64_rescoring_of_top_k(B, oracle_lib, small):
    """top_k poses per ligand rescored in FP64 on the GPU equal the oracle's FP64 score of the
    same descriptors; the final best is the FP64 argmin among them."""
    O = oracle_lib
    p, g, batch = small
    s = S.SMALL.search
    sub = batch.subset(range(12))
    tk = 8
    log("fp64 rescoring top_k=%d" % tk)
    out = run(B, [p], sub, s, top_k=tk)
    check_topk(O, g, s, sub, out, tk)


def test_fp64_rescoring_of_top_k_on_the_largest_ligands(B, oracle_lib, small):
    """The FP64 rescoring with two atoms per lane: ligands of 64, 65, 101 and 128 atoms (even
    and odd counts, so that every rule of the pair split over the atoms is taken) and up to 32
    rotatable bonds; the clash counts, scores and choice equal the oracle's as above."""
    O = oracle_lib
    p, g, _ = small
    ligs = []
    for i, (n, nrot) in enumerate(((64, 6), (65, 9), (101, 20), (128, 32))):
        wl = S.Workload("big%d" % n, 96 + i, 1, 1, (48,), 0.5, 4, ("fixed", n), ("fixed", nrot),
                        S.SMALL.search)
        ligs += S.make_ligands(wl, 0, 1)
    sub = S.batch_from_ligands(ligs)
    tk = 8
    log("fp64 rescoring top_k=%d, n=%s" % (tk, [l.n for l in ligs]))
    out = run(B, [p], sub, S.SMALL.search, top_k=tk)
    check_topk(O, g, S.SMALL.search, sub, out, tk)


def test_graph_replays_match_eager(B, small):
    """EXS_FLAG_GRAPH: the captured launch sequence (counter reset + persistent dock kernel)
    replayed several times, with eager jobs and synchronisations in between, equals the eager
    result every time."""
    p, g, batch = small
    s = S.SMALL.search
    eager = run(B, [p], batch, s, flags=B.EXS_FLAG_PERSISTENT, lpw=2)
    pid = B.exs_load_pocket_grid(p.values, p.spacing, p.origin)
    bid = B.exs_upload_ligands(batch, pocket_ids=[pid])
    L, A = batch.n_ligands, int(batch.atom_offset[-1])
    gp = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, ligands_per_wg=2,
                         flags=B.EXS_FLAG_PERSISTENT | B.EXS_FLAG_GRAPH)
    ep = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, ligands_per_wg=1)
    try:
        for rep in range(3):
            log("graph replay", rep)
            job = B.exs_dock_batch(bid, gp)
            with pytest.raises(B.ExsError):
                B.exs_dock_batch(bid, gp)              # plan held by the unreleased job
            out = B.exs_get_best_poses(job, L, A)
            orient = B.exs_get_orientation_results(job, L, s.n_orient)
            B.exs_release_job(job)
            assert np.array_equal(out["best_score"], eager["best_score"])
            assert np.array_equal(out["coords"], eager["coords"])
            assert np.array_equal(orient["score"], eager["score"])
            assert np.array_equal(orient["desc"]["theta"], eager["desc"]["theta"])
            # eager work and a sync between replays
            job2 = B.exs_dock_batch(bid, ep)
            B.exs_get_best_poses(job2, L, A)
            B.exs_release_job(job2)
    finally:
        B.exs_release_ligands(bid)
        B.exs_unload_pocket(pid)
