"""Seeded input generators: determinism, distributions, geometry (no method arithmetic)."""
import itertools
import math

import numpy as np

import exs_synth as S


def test_separable_grid_equals_direct_formula():
    p = S.make_pocket("small")
    d = S.pocket_grid_values_direct(p.n, p.spacing, p.pseudo_xyz, p.pseudo_w)
    assert np.array_equal(d, p.values)


def test_counter_based_regeneration():
    a = S.make_ligands("batched", 100, 5)
    b = S.make_ligands("batched", 102, 1)[0]
    assert np.array_equal(a[2].xyz, b.xyz) and np.array_equal(a[2].rot, b.rot)
    assert S.pocket_edge("batched", 7) == S.make_pocket("batched", 7).n


def test_ligand_geometry_and_distributions():
    ligs = S.make_ligands("batched", 0, 400)
    ns = np.array([l.n for l in ligs])
    assert ns.min() >= 10 and ns.max() <= 90 and abs(np.median(ns) - 35) <= 3
    for l in ligs[:50]:
        d = np.linalg.norm(l.xyz[l.bonds[:, 0]] - l.xyz[l.bonds[:, 1]], axis=1)
        assert np.allclose(d, 1.5, atol=1e-5)
        deg = np.bincount(l.bonds.reshape(-1), minlength=l.n)
        assert deg.max() <= 4
        for b in l.rot:                                   # rotatable edges are non-terminal
            i, j = l.bonds[b]
            assert deg[i] >= 2 and deg[j] >= 2
        par = {int(c): int(p) for p, c in l.bonds}
        for a in range(2, l.n):                           # 109.5 degrees to the angle reference
            p = par[a]
            r = par[p] if p != 0 else 1
            v1, v2 = l.xyz[r] - l.xyz[p], l.xyz[a] - l.xyz[p]
            ang = math.degrees(math.acos(np.dot(v1, v2) / np.linalg.norm(v1) / np.linalg.norm(v2)))
            assert abs(ang - 109.5) < 1e-3


def test_trace_is_seeded():
    t1 = S.make_trace(50, 100.0)
    t2 = S.make_trace(50, 100.0)
    assert [(r.arrival_s, r.size, r.pocket) for r in t1] == [(r.arrival_s, r.size, r.pocket) for r in t2]
    assert all(1 <= r.size <= 512 for r in t1)
