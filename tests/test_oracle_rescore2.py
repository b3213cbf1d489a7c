"""Pins of the oracle's second-stage score (the fourth step of the method: the first poses of
each ligand's ranked list are rescored with a richer score; the stand-in defined in
oracle/exs_oracle.c): closed forms of each term on hand-built ligands, the exclusions, the
neighbour that defines each dihedral, invariance under rigid motion, and the tie rule of the
selection.  CPU only."""
import math

import numpy as np
import pytest

import exs_synth as S

SIG, EPS, W = 2.0, 0.25, 0.5


class Lig:
    def __init__(self, xyz, bonds, rot=(), types=None):
        self.xyz = np.asarray(xyz, np.float64)
        n = self.xyz.shape[0]
        self.types = np.zeros(n, np.uint8) if types is None else np.asarray(types, np.uint8)
        self.bonds = np.asarray(bonds, np.int32).reshape(-1, 2)
        self.rot = np.asarray(rot, np.int32)


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


@pytest.fixture(scope="module")
def flat(O):
    """A 16^3 x 2 grid of constant value 3.25 (exact in binary): the grid term of n atoms is
    exactly 3.25 n wherever they are."""
    vals = np.full((2, 16, 16, 16), 3.25, np.float32)
    return O.Grid(vals, 0.5, np.full(3, -3.75))


def e2(O, grid, lig, X=None):
    return O.rescore2(grid, lig, lig.xyz if X is None else X, SIG, EPS, W)


@pytest.mark.parametrize("d,contact", [
    (2.0, -EPS),                                   # the well: (s/d)^12 - 2 (s/d)^6 = -1 at d = s
    (1.0, EPS * (4096.0 - 128.0)),                 # d = s/2: 2^12 - 2 * 2^6
    (0.3, EPS * (4096.0 - 128.0)),                 # below s/2 the distance is capped at s/2
    (4.0, EPS * (1.0 / 4096.0 - 2.0 / 64.0)),      # d = 2 s
])
def test_contact_term_closed_form(O, flat, d, contact):
    lig = Lig([[0.0, 0.0, 0.0], [d, 0.0, 0.0]], np.zeros((0, 2)))   # unbonded pair: counted
    e, (grid, cont, tors) = e2(O, flat, lig)
    assert grid == 2 * 3.25 and tors == 0.0
    assert cont == pytest.approx(contact, rel=1e-14, abs=1e-15)
    assert e == pytest.approx(2 * 3.25 + contact, rel=1e-14)


def test_pairs_within_three_bonds_are_excluded(O, flat):
    """A 4-chain has no pair four bonds apart: contact 0 even with atoms on top of each other;
    a 5-chain counts exactly the (0, 4) pair."""
    chain4 = Lig([[0, 0, 0], [0.1, 0, 0], [0.2, 0, 0], [0.0, 0.05, 0]], [[0, 1], [1, 2], [2, 3]])
    assert e2(O, flat, chain4)[1][1] == 0.0
    X = np.array([[0, 0, 0], [1.5, 0, 0], [3.0, 0, 0], [4.5, 0, 0], [2.0, 0, 0]], float)
    chain5 = Lig(X, [[0, 1], [1, 2], [2, 3], [3, 4]])
    # (0, 4) at distance 2.0 = s -> -eps; nothing else
    assert e2(O, flat, chain5)[1][1] == pytest.approx(-EPS, rel=1e-14)


def dihedral_chain(phi, extra=None):
    """Atoms 0-1-2-3, bond 1-2 along x; atom 0 in the xy plane, atom 3 turned by phi about x:
    dihedral 0-1-2-3 = phi."""
    X = [[-0.5, 1.0, 0.0], [0.0, 0.0, 0.0], [1.5, 0.0, 0.0],
         [2.0, math.cos(phi), math.sin(phi)]]
    bonds = [[0, 1], [1, 2], [2, 3]]
    if extra is not None:
        X.append(extra)
        bonds.append([1, 4])
    return X, bonds


@pytest.mark.parametrize("phi,value", [(0.0, 2 * W), (math.pi / 3, 0.0), (math.pi / 2, W),
                                       (math.pi, 0.0), (2 * math.pi / 3, 2 * W),
                                       (math.pi / 4, W * (1 + math.cos(3 * math.pi / 4)))])
def test_torsion_term_closed_form(O, flat, phi, value):
    X, bonds = dihedral_chain(phi)
    for rot_bond in (1,):
        lig = Lig(X, bonds, [rot_bond])
        assert e2(O, flat, lig)[1][2] == pytest.approx(value, abs=1e-12)
    # the same bond listed the other way round
    rev = Lig(X, [[0, 1], [2, 1], [2, 3]], [1])
    assert e2(O, flat, rev)[1][2] == pytest.approx(value, abs=1e-12)
    # not rotatable: no term
    assert e2(O, flat, Lig(X, bonds, []))[1][2] == 0.0


def test_dihedral_uses_the_lowest_index_neighbour(O, flat):
    """Atom 1 has neighbours 0 (dihedral 0 with atom 3) and 4 (dihedral 90 degrees): the term is
    that of atom 0, 2 w; renumbering so that the other neighbour comes first gives w."""
    X, bonds = dihedral_chain(0.0, extra=[-0.5, 0.0, 1.0])
    assert e2(O, flat, Lig(X, bonds, [1]))[1][2] == pytest.approx(2 * W, abs=1e-12)
    perm = [4, 1, 2, 3, 0]                      # swap the labels of atoms 0 and 4
    Xp = [X[perm[i]] for i in range(5)]
    bp = [[perm[a], perm[b]] for a, b in bonds]
    assert e2(O, flat, Lig(Xp, bp, [1]))[1][2] == pytest.approx(W, abs=1e-12)


def test_undefined_dihedral_contributes_nothing(O, flat):
    X = [[-1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.5, 0.0, 0.0], [2.0, 1.0, 0.0]]   # 0, 1, 2 collinear
    assert e2(O, flat, Lig(X, [[0, 1], [1, 2], [2, 3]], [1]))[1][2] == 0.0
    X = [[0.0, 0.0, 0.0], [1.5, 0.0, 0.0]]                                      # no neighbours
    assert e2(O, flat, Lig(X, [[0, 1]], [0]))[1][2] == 0.0


def test_grid_term_reads_the_texel_at_grid_points(O):
    """On the oracle-sized pocket, a one-atom ligand placed on a texel gets that texel exactly."""
    p = S.make_pocket("small")
    g = O.Grid.of(p)
    for (i, j, k, c) in ((0, 0, 0, 0), (47, 3, 20, 1), (10, 47, 47, 3), (23, 24, 25, 2)):
        X = np.array([[p.origin[0] + p.spacing * i, p.origin[1] + p.spacing * j,
                       p.origin[2] + p.spacing * k]])
        lig = Lig(X, np.zeros((0, 2)), [], [c])
        assert e2(O, g, lig)[1][0] == float(p.values[c, k, j, i])


def test_internal_terms_are_invariant_under_rigid_motion(O, flat):
    """Contact and torsion terms depend only on internal geometry: a random rotation and shift
    of a generated ligand leaves them unchanged (the grid term is constant on this grid)."""
    rng = np.random.default_rng(5)
    for lig in S.make_ligands("scale", 0, 6):
        lig4 = Lig(lig.xyz.astype(np.float64), lig.bonds, lig.rot, lig.types % 2)
        e_a, parts_a = e2(O, flat, lig4)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        a, b, c, d = q
        R = np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                      [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                      [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])
        X = lig4.xyz @ R.T + rng.normal(size=3)
        e_b, parts_b = e2(O, flat, lig4, X)
        assert parts_b[1] == pytest.approx(parts_a[1], rel=1e-10, abs=1e-10)
        assert parts_b[2] == pytest.approx(parts_a[2], rel=1e-10, abs=1e-10)
        assert e_b == pytest.approx(e_a, rel=1e-10)


def test_stage2_selection_takes_the_lowest_then_the_earlier(O):
    assert O.stage2_best([3.0, 1.0, 2.0]) == 1
    assert O.stage2_best([1.0, 1.0, 0.5, 0.5]) == 2
    assert O.stage2_best([7.0]) == 0
