"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Each test fixes a property of the method that does not come from the oracle
itself: texel values on grid nodes, multilinear fields (which trilinear
interpolation reproduces exactly), hand-built molecular geometry with known
distances, Rodrigues rotations about coordinate axes, an independent rotation
library (scipy) for the Fibonacci orientations and for exhaustive pose
enumeration, and exact-arithmetic ramps that expose the candidate order and the
tie rule.  Paper reference: Sec. 3.1 ("The dock and score algorithm").
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import exs_synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class Lig:
    def __init__(self, xyz, types, bonds, rot=()):
        self.xyz = np.asarray(xyz, np.float32)
        self.types = np.asarray(types, np.uint8)
        self.bonds = np.asarray(bonds, np.int32).reshape(-1, 2)
        self.rot = np.asarray(rot, np.int32)


def fit_types(lig, channels):
    return Lig(lig.xyz, lig.types % channels, lig.bonds, lig.rot)


def grid_of(O, values, h):
    n = values.shape[-1]
    return O.Grid(values, h, [-h * (n - 1) / 2.0] * 3)


def params(O, K=4, S_=8, P=1, T=1, **kw):
    return O.Params(K, S_, P, T, **kw)


# ------------------------------------------------------------------------------------------------
# Trilinear grid term
# ------------------------------------------------------------------------------------------------

def test_grid_aligned_atom_returns_texel_exactly(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(1)
    n, c, h = 7, 3, 0.375
    vals = rng.normal(size=(c, n, n, n)).astype(np.float32)
    g = grid_of(O, vals, h)
    o = -h * (n - 1) / 2.0
    pts = [(i, j, k) for i in (0, n - 1) for j in (0, n - 1) for k in (0, n - 1)]   # corners
    pts += [(0, 3, 5), (n - 1, 2, 0), (3, n - 1, 4), (1, 2, 3), (5, 5, 5)]          # faces, interior
    for (i, j, k) in pts:
        for ch in range(c):
            p = (o + h * i, o + h * j, o + h * k)
            assert O.grid_value(g, ch, p) == float(vals[ch, k, j, i])


def test_multilinear_field_reproduced(oracle_lib):
    """V = a + b i + c j + d k + e ij + f jk + g ik + m ijk is reproduced exactly by trilinear."""
    O = oracle_lib
    n, h = 8, 0.5
    coef = [(3, 5, -7, 11, 2, -3, 4, 1), (-2, 1, 9, -4, -1, 2, 3, -2)]
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")

    def field(cf, x, y, z):
        a, b, c, d, e, f, g_, m = cf
        return a + b * x + c * y + d * z + e * x * y + f * y * z + g_ * x * z + m * x * y * z

    vals = np.zeros((2, n, n, n), np.float32)
    for ch, cf in enumerate(coef):
        vals[ch] = np.transpose(field(cf, i, j, k), (2, 1, 0))   # [z][y][x]
    g = grid_of(O, vals, h)
    o = -h * (n - 1) / 2.0
    rng = np.random.default_rng(2)
    for _ in range(200):
        u = rng.uniform(0, n - 1, size=3)
        p = o + h * u
        for ch, cf in enumerate(coef):
            want = field(cf, *u)
            got = O.grid_value(g, ch, p)
            assert abs(got - want) <= 1e-9 * max(1.0, abs(want))


def test_outside_points_clamp_to_face(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(3)
    n, h = 6, 0.5
    vals = rng.normal(size=(1, n, n, n)).astype(np.float32)
    g = grid_of(O, vals, h)
    o = -h * (n - 1) / 2.0
    hi = o + h * (n - 1)
    assert O.grid_value(g, 0, (hi + 3.0, hi + 1.0, hi + 7.0)) == float(vals[0, n - 1, n - 1, n - 1])
    assert O.grid_value(g, 0, (o - 3.0, o - 1.0, o - 0.1)) == float(vals[0, 0, 0, 0])
    for _ in range(50):
        p = rng.uniform(o, hi, size=3)
        q = p.copy(); q[0] = hi + rng.uniform(0.1, 5.0)
        r = p.copy(); r[0] = hi
        assert abs(O.grid_value(g, 0, q) - O.grid_value(g, 0, r)) < 1e-15
        q = p.copy(); q[2] = o - rng.uniform(0.1, 5.0)
        r = p.copy(); r[2] = o
        assert abs(O.grid_value(g, 0, q) - O.grid_value(g, 0, r)) < 1e-15


def test_upper_face_reads_stay_inside_the_cell(oracle_lib):
    """On the upper face (u = N-1) the cell is N-2 with f = 1: no texel past the face is read
    (an infinite texel right after the face row would turn 0 * inf into NaN)."""
    O = oracle_lib
    n, h = 5, 0.5
    vals = np.ones((1, n, n, n), np.float32)
    vals[0, 0, 1, 0] = np.inf                      # z=0, y=1, x=0: the word after row y=0
    g = grid_of(O, vals, h)
    o = -h * (n - 1) / 2.0
    assert O.grid_value(g, 0, (o + h * (n - 1), o, o)) == 1.0
    assert O.grid_value(g, 0, (o + h * (n - 1) + 1.0, o - 1.0, o)) == 1.0


def test_channel_selection_and_delta_texel(oracle_lib):
    O = oracle_lib
    n, c, h = 5, 4, 0.5
    vals = np.zeros((c, n, n, n), np.float32)
    vals[2, 3, 1, 2] = 1.0   # channel 2, z=3, y=1, x=2
    g = grid_of(O, vals, h)
    o = -h * (n - 1) / 2.0
    node = np.array([o + 2 * h, o + 1 * h, o + 3 * h])
    for ch in range(c):
        assert O.grid_value(g, ch, node) == (1.0 if ch == 2 else 0.0)
    assert O.grid_value(g, 2, node + [h / 2, 0, 0]) == 0.5
    assert O.grid_value(g, 2, node + [0, -h / 2, 0]) == 0.5
    assert O.grid_value(g, 2, node + [h / 2, h / 2, -h / 2]) == 0.125
    assert O.grid_value(g, 2, node + [h / 4, 0, 3 * h / 4]) == 0.75 * 0.25


# ------------------------------------------------------------------------------------------------
# Exclusions and clash term
# ------------------------------------------------------------------------------------------------

def chain_bonds(n):
    return np.array([[a, a + 1] for a in range(n - 1)], np.int32)


@pytest.mark.parametrize("n", [4, 5, 6, 8, 10])
def test_chain_exclusion_counts(oracle_lib, n):
    d = oracle_lib.bond_distances(n, chain_bonds(n))
    iu = np.triu_indices(n, 1)
    non_excluded = int(np.sum(d[iu] >= 4))
    assert non_excluded == math.comb(n, 2) - (3 * n - 6)
    assert d[0, n - 1] == n - 1


def test_disconnected_atoms_are_not_excluded(oracle_lib):
    d = oracle_lib.bond_distances(4, np.array([[0, 1], [2, 3]], np.int32))
    assert d[0, 2] == -1 and d[1, 3] == -1 and d[0, 1] == 1


def _golden_chain():
    with open(os.path.join(GOLDEN, "chain_geometry.json")) as f:
        return json.load(f)


def planar_chain(n, cis):
    """Planar 5-chain with 1.5 A bonds and 109.5 degree angles, all-cis or all-trans."""
    half = math.radians(109.5) / 2
    if not cis:  # zig-zag
        return np.array([[k * 1.5 * math.sin(half), (k % 2) * 1.5 * math.cos(half), 0.0]
                         for k in range(n)])
    gamma = math.pi - math.radians(109.5)          # central angle of the circle through the atoms
    R = 1.5 / (2 * math.sin(gamma / 2))
    return np.array([[R * math.cos(k * gamma), R * math.sin(k * gamma), 0.0] for k in range(n)])


def test_chain_geometry_closed_forms():
    gold = _golden_chain()
    t = planar_chain(5, cis=False)
    c = planar_chain(5, cis=True)
    assert abs(np.linalg.norm(t[0] - t[2]) - gold["d13"]) < 1e-6
    assert abs(np.linalg.norm(t[0] - t[4]) - gold["d15_trans"]) < 1e-6
    assert abs(np.linalg.norm(c[0] - c[4]) - gold["d15_cis"]) < 1e-6


@pytest.mark.parametrize("penalty", [1.0, 2.5])
def test_trans_cis_clash_counts(oracle_lib, penalty):
    O = oracle_lib
    g = grid_of(O, np.zeros((1, 4, 4, 4), np.float32), 0.5)
    prm = params(O, clash_penalty=penalty)
    for cis, want in ((False, 0), (True, 1)):
        X = planar_chain(5, cis)
        e, cl, am = O.score(g, prm, X, np.zeros(5, np.uint8), chain_bonds(5))
        assert cl == want and am == 0
        assert e == penalty * want


def test_clash_cutoff_is_strict(oracle_lib):
    O = oracle_lib
    g = grid_of(O, np.zeros((1, 4, 4, 4), np.float32), 0.5)
    prm = params(O)
    X = np.array([[0, 0, 0], [9, 9, 9], [19, 9, 9], [29, 9, 9], [2.0, 0, 0]], float)
    e, cl, am = O.score(g, prm, X, np.zeros(5, np.uint8), chain_bonds(5))
    assert (e, cl, am) == (0.0, 0, 1)                 # d = 2.0 exactly: not a clash, ambiguous
    X[4, 0] = 1.999
    e, cl, am = O.score(g, prm, X, np.zeros(5, np.uint8), chain_bonds(5))
    assert (e, cl, am) == (1.0, 1, 0)
    X[4, 0] = 0.5                                      # bonded neighbours never clash
    X[1] = [0.1, 0, 0]
    e, cl, am = O.score(g, prm, X, np.zeros(5, np.uint8), chain_bonds(5))
    assert cl == 1


# ------------------------------------------------------------------------------------------------
# Rotations and topology
# ------------------------------------------------------------------------------------------------

def test_rodrigues_axis_closed_form(oracle_lib):
    O = oracle_lib
    X = np.array([[0, 0, 0], [0, 0, 1], [1, 0, 1], [2, 0, 3]], float)   # axis 0 -> 1 is +z
    mv = np.array([0, 0, 1, 1], np.uint8)
    Y = O.rotate_about_bond(X, 0, 1, mv, math.pi / 2)
    assert np.allclose(Y[2], [0, 1, 1], atol=1e-15) and np.allclose(Y[3], [0, 2, 3], atol=1e-15)
    Y = O.rotate_about_bond(X, 0, 1, mv, math.pi)
    assert np.allclose(Y[2], [-1, 0, 1], atol=1e-15)
    assert np.array_equal(Y[:2], X[:2])
    # reversed axis turns the other way
    Y = O.rotate_about_bond(X, 1, 0, mv, math.pi / 2)
    assert np.allclose(Y[2], [0, -1, 1], atol=1e-15)


@pytest.mark.parametrize("K", [1, 7, 64, 256])
def test_fibonacci_orientations(oracle_lib, K):
    O = oracle_lib
    golden = math.pi * (3 - math.sqrt(5))
    for k in range(K):
        R = O.orientation(k, K)
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14
        zk = 1 - (2 * k + 1) / K
        beta, phi = math.acos(zk), k * golden
        want = [math.sin(beta) * math.cos(phi), math.sin(beta) * math.sin(phi), zk]
        assert np.allclose(R @ [0, 0, 1], want, atol=1e-14)
        ref = Rotation.from_euler("ZY", [phi, beta]).as_matrix()
        assert np.allclose(R, ref, atol=1e-13)


def test_moving_sets_closed_forms(oracle_lib):
    O = oracle_lib
    u, v, m = O.rot_topology(5, chain_bonds(5), np.array([1], np.int32))
    assert (u[0], v[0]) == (1, 2) and m[0].tolist() == [False, False, False, True, True]
    bonds = np.array([[2, 1], [0, 1], [3, 2]], np.int32)              # listed reversed
    u, v, m = O.rot_topology(4, bonds, np.array([0], np.int32))
    assert (u[0], v[0]) == (1, 2) and m[0].tolist() == [False, False, False, True]
    branch = np.array([[0, 1], [1, 2], [1, 3], [3, 4], [3, 5]], np.int32)
    u, v, m = O.rot_topology(6, branch, np.array([2], np.int32))
    assert (u[0], v[0]) == (1, 3) and np.flatnonzero(m[0]).tolist() == [4, 5]
    ring = np.array([[0, 1], [1, 2], [2, 0], [2, 3]], np.int32)
    with pytest.raises(ValueError):
        O.rot_topology(4, ring, np.array([0], np.int32))
    u, v, m = O.rot_topology(4, ring, np.array([3], np.int32))
    assert (u[0], v[0]) == (2, 3) and not m[0].any()


@pytest.fixture(scope="module")
def small_case(oracle_lib):
    p = S.make_pocket("small")
    return oracle_lib.Grid.of(p), S.make_ligands("small", 0, 3)


def test_bond_geometry_preserved_by_search(oracle_lib, small_case):
    O = oracle_lib
    g, ligs = small_case
    prm = O.Params.of(S.SMALL.search)
    for lig in ligs:
        r = O.dock_ligand(g, prm, lig, coords=True)
        X0 = lig.xyz.astype(np.float64)
        d = O.bond_distances(lig.n, lig.bonds)
        pairs = np.argwhere((d >= 1) & (d <= 2))        # bond lengths and bond angles
        ref = np.linalg.norm(X0[pairs[:, 0]] - X0[pairs[:, 1]], axis=1)
        for k in range(prm.n_orient):
            X = r["coords"][k]
            got = np.linalg.norm(X[pairs[:, 0]] - X[pairs[:, 1]], axis=1)
            assert np.max(np.abs(got - ref)) < 1e-12


def test_full_turn_leaves_score_unchanged(oracle_lib, small_case):
    O = oracle_lib
    g, ligs = small_case
    prm = O.Params.of(S.SMALL.search, n_orient=1)
    checked = 0
    for lig in ligs:
        X = O.pose_from_desc(g, O.Params.of(S.SMALL.search), lig, 5, [0] * len(lig.rot), [0, 0, 0])
        e0, _, am = O.score(g, prm, X, lig.types, lig.bonds)
        if am:
            continue
        u, v, m = O.rot_topology(lig.n, lig.bonds, lig.rot)
        for b in range(len(lig.rot)):
            Y = O.rotate_about_bond(X, u[b], v[b], m[b], 2 * math.pi)
            assert np.max(np.abs(Y - X)) < 1e-13
            e1, _, _ = O.score(g, prm, Y, lig.types, lig.bonds)
            assert abs(e1 - e0) < 1e-12 * max(1, abs(e0))
            checked += 1
    assert checked > 0


@pytest.mark.parametrize("wl", ["small", "scale"])
def test_descriptor_rebuilds_incremental_pose(oracle_lib, wl):
    """C.10 order independence: c + step*tau + R_k FK_theta(X0) equals the searched pose."""
    O = oracle_lib
    w = S.WORKLOADS[wl]
    g = O.Grid.of(S.make_pocket("small"))
    prm = O.Params.of(w.search, n_orient=8, passes=2)
    ligs = [fit_types(l, 4) for l in S.make_ligands(wl, 0, 12) if len(l.rot) >= 2][:3]
    for lig in ligs:
        r = O.dock_ligand(g, prm, lig, coords=True)
        for k in range(prm.n_orient):
            X = O.pose_from_desc(g, prm, lig, k, r["theta"][k], r["tau"][k])
            assert np.max(np.abs(X - r["coords"][k])) < 1e-12
            e, _, am = O.score(g, prm, X, lig.types, lig.bonds)
            assert abs(e - r["score"][k]) <= 1e-9 * max(1, abs(e)) + prm.clash_penalty * am


# ------------------------------------------------------------------------------------------------
# Search
# ------------------------------------------------------------------------------------------------

def test_bruteforce_three_atom_ligands(oracle_lib, small_case):
    """0 rotatable bonds, one pass: the greedy offset sweep is exhaustive over K x 27 poses."""
    O = oracle_lib
    g, _ = small_case
    K = 16
    prm = O.Params(K, 8, 1, 27)
    centre = np.zeros(3)
    golden = math.pi * (3 - math.sqrt(5))
    half = math.radians(109.5) / 2
    base = np.array([[0, 0, 0], [1.5, 0, 0],
                     [1.5 * math.cos(2 * half), 1.5 * math.sin(2 * half), 0]])
    rng = np.random.default_rng(5)
    for trial in range(6):
        xyz = (base + rng.normal(scale=0.05, size=3)).astype(np.float32)
        lig = Lig(xyz, rng.integers(0, 4, 3), [[0, 1], [0, 2]])
        r = O.dock_ligand(g, prm, lig)
        X0 = xyz.astype(np.float64) - xyz.astype(np.float64).mean(axis=0)
        best = None
        for k in range(K):
            zk = 1 - (2 * k + 1) / K
            Rk = Rotation.from_euler("ZY", [k * golden, math.acos(zk)]).as_matrix()
            P = centre + X0 @ Rk.T
            order = [13] + [o for o in range(27) if o != 13]        # keep first
            for rank, o in enumerate(order):
                d = 0.5 * np.array([o // 9 - 1, (o // 3) % 3 - 1, o % 3 - 1])
                e, _, _ = O.score(g, prm, P + d, lig.types, lig.bonds)
                key = (e, k, rank)
                if best is None or key[0] < best[0][0] - 1e-12:
                    best = (key, o)
        (e, k, rank), o = best
        assert abs(r["best_score"] - e) < 1e-9
        assert r["best_k"] == k
        assert r["tau"][k].tolist() == [o // 9 - 1, (o // 3) % 3 - 1, o % 3 - 1]


def test_bruteforce_four_atom_one_bond(oracle_lib, small_case):
    """One rotatable bond, T = 1, one pass: greedy is exhaustive over K x S poses."""
    O = oracle_lib
    g, _ = small_case
    K, Sn = 16, 16
    prm = O.Params(K, Sn, 1, 1)
    golden = math.pi * (3 - math.sqrt(5))
    rng = np.random.default_rng(6)
    for trial in range(6):
        xyz = planar_chain(4, cis=False) + rng.normal(scale=0.02, size=(4, 3))
        lig = Lig(xyz.astype(np.float32), rng.integers(0, 4, 4), chain_bonds(4), [1])
        r = O.dock_ligand(g, prm, lig)
        X0 = lig.xyz.astype(np.float64) - lig.xyz.astype(np.float64).mean(axis=0)
        best = None
        for k in range(K):
            zk = 1 - (2 * k + 1) / K
            Rk = Rotation.from_euler("ZY", [k * golden, math.acos(zk)]).as_matrix()
            P = X0 @ Rk.T
            axis = P[2] - P[1]
            axis /= np.linalg.norm(axis)
            for s in range(Sn):          # s = 0 is the keep candidate, first in order
                Q = P.copy()
                Q[3] = P[2] + Rotation.from_rotvec(axis * (2 * math.pi * s / Sn)).apply(P[3] - P[2])
                e, _, _ = O.score(g, prm, Q, lig.types, lig.bonds)
                if best is None or e < best[0] - 1e-12:
                    best = (e, k, s)
        e, k, s = best
        assert abs(r["best_score"] - e) < 1e-9
        assert r["best_k"] == k and int(r["theta"][k][0]) == s


def test_trajectory_monotone_and_final_is_min(oracle_lib, small_case):
    O = oracle_lib
    g, _ = small_case
    prm = O.Params.of(S.SCALE.search, n_orient=8)
    for lig in S.make_ligands("scale", 0, 3):
        lig = fit_types(lig, 4)
        r = O.dock_ligand(g, prm, lig, trace_cap=64)
        for k in range(prm.n_orient):
            tr = r["trace"][k]
            tr = tr[~np.isnan(tr)]
            assert tr[0] == r["start"][k]
            assert np.all(np.diff(tr) <= 0)
            assert tr[-1] == r["score"][k] == r["min_cand"][k]
        assert r["best_k"] == int(np.argmin(r["score"]))


def _one_atom_on_ramp(O, axis, sign, passes=2):
    n, h = 12, 0.5
    idx = np.arange(n, dtype=np.float32)
    shape = [1, 1, 1]
    shape[2 - axis] = n                           # values are [z][y][x]
    ramp = (sign * idx).reshape(shape)
    vals = np.broadcast_to(ramp, (n, n, n)).astype(np.float32)[None]
    g = grid_of(O, np.ascontiguousarray(vals), h)
    lig = Lig([[0.25, -1.0, 3.0]], [0], np.zeros((0, 2)))
    return O.dock_ligand(g, O.Params(1, 8, passes, 27), lig)


def test_offset_order_and_tie_rule_on_exact_ramps(oracle_lib):
    """Exact arithmetic (one atom on grid nodes, dyadic spacing): ties go to the first
    candidate in order (a,b,c) with a slowest, keep before all."""
    O = oracle_lib
    r = _one_atom_on_ramp(O, axis=0, sign=+1.0)      # lower x better: a=-1, ties -> (-1,-1,-1)
    assert r["tau"][0].tolist() == [-2, -2, -2]
    r = _one_atom_on_ramp(O, axis=0, sign=-1.0)      # higher x better: first is (1,-1,-1)
    assert r["tau"][0].tolist() == [2, -2, -2]
    r = _one_atom_on_ramp(O, axis=2, sign=-1.0)      # higher z better: first is (-1,-1,1)
    assert r["tau"][0].tolist() == [-2, -2, 2]
    r = _one_atom_on_ramp(O, axis=1, sign=-1.0, passes=1)
    assert r["tau"][0].tolist() == [-1, 1, -1]
    assert r["near_tie"][0]                          # exact ties are flagged


def test_constant_grid_keeps_pose_and_lowest_orientation(oracle_lib):
    O = oracle_lib
    g = grid_of(O, np.zeros((1, 6, 6, 6), np.float32), 0.5)
    lig = Lig(planar_chain(4, cis=False), [0, 0, 0, 0], chain_bonds(4), [1])
    r = O.dock_ligand(g, O.Params(8, 8, 2, 27), lig)
    assert np.all(r["tau"] == 0) and np.all(r["theta"] == 0)
    assert r["best_k"] == 0 and r["best_score"] == 0.0 and r["near_tie"].all()


def test_oracle_regression_fixture(oracle_lib):
    """Guards the oracle against accidental change (fixture written by make_golden.py)."""
    O = oracle_lib
    with open(os.path.join(GOLDEN, "oracle_small.json")) as f:
        gold = json.load(f)
    g = O.Grid.of(S.make_pocket("small"))
    prm = O.Params.of(S.SMALL.search)
    for entry in gold["ligands"]:
        lig = S.make_ligands("small", entry["index"], 1)[0]
        r = O.dock_ligand(g, prm, lig)
        assert r["best_k"] == entry["best_k"]
        assert np.allclose(r["score"], entry["score"], rtol=1e-12, atol=1e-12)
        assert r["theta"].tolist() == entry["theta"]


# ------------------------------------------------------------------------------------------------
# Ranking of the final poses: RMSD clustering, leaders first (Sec. 3.1, third step)


def test_rmsd_closed_forms(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(3)
    X = rng.normal(size=(7, 3))
    assert O.rmsd(X, X) == 0.0
    t = np.array([1.0, 2.0, 2.0])
    assert abs(O.rmsd(X, X + t) - 3.0) < 1e-12                  # a translation moves every atom by |t|
    R = np.diag([-1.0, -1.0, 1.0])                              # half turn about z
    P = np.array([[2.0, 0.0, 5.0], [0.0, 1.0, -1.0]])
    # distances 2*2 and 2*1 -> sqrt((16 + 4) / 2)
    assert abs(O.rmsd(P, P @ R.T) - np.sqrt(10.0)) < 1e-12
    Y = rng.normal(size=(7, 3))
    assert O.rmsd(X, Y) == O.rmsd(Y, X)


def test_rank_poses_on_a_line(oracle_lib):
    """Rigid copies of a 2-atom pose 1 A apart along x, better first: leaders every 3 A, a pose
    exactly 3 A from a leader starts its own cluster (similar means below the threshold)."""
    O = oracle_lib
    K = 8
    poses = np.zeros((K, 2, 3))
    poses[:, 1, 1] = 1.5
    poses[:, :, 0] += np.arange(K)[:, None]
    r = O.rank_poses(poses, np.arange(K, dtype=float), 3.0)
    assert r["leader"].tolist() == [True, False, False, True, False, False, True, False]
    assert r["order"].tolist() == [0, 3, 6, 1, 2, 4, 5, 7]
    assert r["n_leaders"] == 3 and r["amb_rmsd"] == 2
    r = O.rank_poses(poses, np.arange(K, dtype=float), 3.0 + 1e-9)
    assert r["leader"].tolist() == [True, False, False, False, True, False, False, False]
    # the scores, not the indices, decide who leads: reverse them
    r = O.rank_poses(poses, -np.arange(K, dtype=float), 3.0)
    assert r["order"][0] == K - 1 and r["leader"][K - 1] and r["leader"][K - 4]


def _check_greedy_leaders(O, poses, scores, thr, r):
    """The output of the ranking is fixed by these properties (the first pose where two
    outputs differ would contradict one of them): a permutation; leaders listed by score
    and then the others by score; every leader at RMSD >= thr from every better leader;
    every other pose below thr from some better leader."""
    K = len(scores)
    order = r["order"]
    assert sorted(order.tolist()) == list(range(K))
    by = sorted(range(K), key=lambda k: (scores[k], k))
    pos = {k: i for i, k in enumerate(by)}
    lead = [k for k in by if r["leader"][k]]
    rest = [k for k in by if not r["leader"][k]]
    assert order.tolist() == lead + rest
    for k in by:
        better = [q for q in lead if pos[q] < pos[k]]
        d = [O.rmsd(poses[k], poses[q]) for q in better]
        if r["leader"][k]:
            assert all(x >= thr for x in d)
        else:
            assert any(x < thr for x in d)


def test_rank_poses_properties_on_random_poses(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(11)
    for trial in range(6):
        K, n = int(rng.integers(5, 60)), int(rng.integers(1, 12))
        base = rng.normal(size=(n, 3)) * 2.0
        poses = base[None] + rng.normal(size=(K, 1, 3)) * rng.uniform(1.0, 4.0) \
            + rng.normal(size=(K, n, 3)) * 0.5
        scores = np.round(rng.normal(size=K), 1)                 # ties on purpose
        thr = float(rng.uniform(0.5, 5.0))
        r = O.rank_poses(poses, scores, thr)
        _check_greedy_leaders(O, poses, scores, thr, r)


def test_rank_poses_special_cases(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(5)
    K, n = 40, 6
    poses = rng.normal(size=(K, n, 3)) * 3.0
    scores = rng.normal(size=K)
    scores[7] = scores[3]                                        # a tie: index 3 goes first
    by = np.lexsort((np.arange(K), scores))
    r = O.rank_poses(poses, scores, 0.0)                         # nothing is similar
    assert r["n_leaders"] == K and r["order"].tolist() == by.tolist()
    r = O.rank_poses(poses, scores, np.inf)                      # everything is similar
    assert r["n_leaders"] == 1 and r["order"].tolist() == by.tolist()
    same = np.repeat(poses[:1], K, axis=0)
    r = O.rank_poses(same, scores, 1e-9)                         # identical poses: one cluster
    assert r["n_leaders"] == 1 and r["order"].tolist() == by.tolist()
    s2 = scores.copy()
    s2[[0, 9]] = np.nan                                          # NaN scores rank last
    r = O.rank_poses(poses, s2, 0.0)
    assert r["order"][-2:].tolist() == [0, 9]


# ------------------------------------------------------------------------------------------------
# Unfolding of the input conformation (Sec. 3.1, first step)


def test_distance_sum_closed_forms(oracle_lib):
    O = oracle_lib
    a = 1.7
    tri = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * np.sqrt(3) / 2, 0]])
    assert abs(O.distance_sum(tri) - 3 * a) < 1e-12
    tet = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)   # edge 2 sqrt 2
    assert abs(O.distance_sum(tet) - 6 * 2 * np.sqrt(2)) < 1e-12
    rng = np.random.default_rng(2)
    X = rng.normal(size=(9, 3))
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    assert abs(O.distance_sum(X @ Q.T + [3, -1, 2]) - O.distance_sum(X)) < 1e-10
    assert O.distance_sum(X[:1]) == 0.0


class _Lig:
    def __init__(self, xyz, bonds, rot):
        self.xyz = np.asarray(xyz, np.float32)
        self.types = np.zeros(len(xyz), np.uint8)
        self.bonds = np.asarray(bonds, np.int32)
        self.rot = np.asarray(rot, np.int32)


def test_unfold_turns_an_all_cis_chain_all_trans(oracle_lib):
    """A planar all-cis 5-chain with its two inner bonds rotatable unfolds to the planar
    zig-zag: every distance is the all-trans closed form (d15 = 2 d13)."""
    O = oracle_lib
    gold = _golden_chain()
    cis = planar_chain(5, cis=True)
    trans = planar_chain(5, cis=False)
    lig = _Lig(cis, chain_bonds(5), [1, 2])
    r = O.unfold_ligand(lig, 8, 2)
    X = r["xyz"]
    D = np.linalg.norm(X[:, None] - X[None], axis=-1)
    T = np.linalg.norm(trans[:, None] - trans[None], axis=-1)
    assert np.abs(D - T).max() < 1e-5                      # the input is float32
    assert abs(D[0, 4] - gold["d15_trans"]) < 1e-5
    assert r["turns"][0].tolist() == [4, 4]                  # half turns, then nothing to gain
    assert r["turns"][1].tolist() == [0, 0]
    assert abs(O.distance_sum(X) - O.distance_sum(trans)) < 1e-4


def test_unfold_keeps_geometry_and_never_shrinks(oracle_lib):
    O = oracle_lib
    for lig in S.make_ligands("batched", 3, 6):
        X0 = lig.xyz.astype(np.float64)
        r = O.unfold_ligand(lig, 16, 2)
        X = r["xyz"]
        assert O.distance_sum(X) >= O.distance_sum(X0) - 1e-9
        bl0 = np.linalg.norm(X0[lig.bonds[:, 0]] - X0[lig.bonds[:, 1]], axis=1)
        bl = np.linalg.norm(X[lig.bonds[:, 0]] - X[lig.bonds[:, 1]], axis=1)
        assert np.abs(bl - bl0).max() < 1e-9
        _, _, moving = O.rot_topology(lig.n, lig.bonds, lig.rot)
        still = ~moving.any(axis=0) if len(lig.rot) else np.ones(lig.n, bool)
        assert np.array_equal(X[still], X0[still])         # atom 0's side never moves


def test_unfold_converges_to_a_single_bond_optimum(oracle_lib):
    """After enough passes no single turn of any rotatable bond increases the distance sum."""
    O = oracle_lib
    S_ = 16
    for lig in S.make_ligands("batched", 4, 3):
        r = O.unfold_ligand(lig, S_, 40)
        X = r["xyz"]
        assert not r["turns"][-1].any()
        u, v, moving = O.rot_topology(lig.n, lig.bonds, lig.rot)
        D = O.distance_sum(X)
        for b in range(len(lig.rot)):
            for s in range(1, S_):
                Y = O.rotate_about_bond(X, u[b], v[b], moving[b], 2 * np.pi * s / S_)
                assert O.distance_sum(Y) <= D + 1e-9


def test_unfold_near_tie_band_is_per_changed_distance(oracle_lib):
    """The near-tie band of an unfolding decision is tol * m * (n - m) (m turning atoms): on the
    all-cis 5-chain the first decision (bond 1-2, m = 2, 6 changed distances) is flagged for a
    tol just above gap / 6 and not for one just below, where gap is the distance-sum margin of
    the kept turn over the next best, computed here from the distances themselves."""
    O = oracle_lib
    cis = planar_chain(5, cis=True)
    lig = _Lig(cis, chain_bonds(5), [1])
    X = cis.astype(np.float32).astype(np.float64)
    moving = np.array([False, False, False, True, True])
    axis = X[2] - X[1]
    axis /= np.linalg.norm(axis)
    sums = []
    for s in range(8):
        a = 2 * np.pi * s / 8
        Y = X.copy()
        for i in np.nonzero(moving)[0]:
            r = X[i] - X[2]
            Y[i] = X[2] + r * np.cos(a) + np.cross(axis, r) * np.sin(a) + axis * axis.dot(r) * (1 - np.cos(a))
        D = np.linalg.norm(Y[:, None] - Y[None], axis=-1)
        sums.append(D[np.triu_indices(5, 1)].sum())
    srt = sorted(sums, reverse=True)
    gap = srt[0] - srt[1]
    assert gap > 1e-3
    assert O.unfold_ligand(lig, 8, 1, tol=gap / 6 * 1.01)["near_ties"] == 1
    assert O.unfold_ligand(lig, 8, 1, tol=gap / 6 * 0.99)["near_ties"] == 0
    assert O.unfold_band(5, 2, 1.0) == 6.0
