"""C ABI checks that need no GPU: the library loads, exports every declared entry
point, and its host-side topology packing (validation, exclusion and moving
masks) agrees with closed forms and with the oracle's independent BFS."""
import os
import re

import numpy as np
import pytest

import exs_synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_2110_11644_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2110_11644_amd import build
        build.build()
    binding.lib()
    return binding


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "exs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(exs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(B):
    decl = declared_symbols()
    assert len(decl) >= 10
    L = B.lib()
    for name in decl:
        assert hasattr(L, name), name
    assert set(decl) == set(B.SYMBOLS)
    assert "gfx950" in B.exs_version()


class Lig:
    def __init__(self, xyz, types, bonds, rot=()):
        self.xyz = np.asarray(xyz, np.float32)
        self.types = np.asarray(types, np.uint8)
        self.bonds = np.asarray(bonds, np.int32).reshape(-1, 2)
        self.rot = np.asarray(rot, np.int32)


def chain(n, rot=()):
    return Lig(np.arange(3 * n, dtype=np.float32).reshape(n, 3), np.zeros(n),
               [[a, a + 1] for a in range(n - 1)], rot)


def test_chain_exclusions_closed_form(B):
    for n in (4, 5, 8, 40, 128):
        t = B.exs_pack_topology(chain(n), 1)
        ex = t["excl"]
        assert ex.shape == (n, n)
        i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        assert np.array_equal(ex, np.abs(i - j) <= 3)


def test_moving_sets_closed_form(B):
    t = B.exs_pack_topology(chain(6, rot=[1, 3]), 1)
    assert t["rot_u"].tolist() == [1, 3] and t["rot_v"].tolist() == [2, 4]
    assert np.flatnonzero(t["moving"][0]).tolist() == [3, 4, 5]
    assert np.flatnonzero(t["moving"][1]).tolist() == [5]
    rev = Lig(np.arange(12.0).reshape(4, 3), np.zeros(4), [[2, 1], [0, 1], [3, 2]], [0])
    t = B.exs_pack_topology(rev, 1)
    assert (t["rot_u"][0], t["rot_v"][0]) == (1, 2)
    assert np.flatnonzero(t["moving"][0]).tolist() == [3]


def test_packing_matches_oracle_bfs(B, oracle_lib):
    O = oracle_lib
    for lig in S.make_ligands("batched", 0, 40):
        t = B.exs_pack_topology(lig, 8)
        d = O.bond_distances(lig.n, lig.bonds)
        assert np.array_equal(t["excl"], (d >= 0) & (d <= 3))
        u, v, m = O.rot_topology(lig.n, lig.bonds, lig.rot)
        assert np.array_equal(t["rot_u"], u) and np.array_equal(t["rot_v"], v)
        assert np.array_equal(t["moving"], m)


@pytest.mark.parametrize("case", ["ring", "type", "bond_index", "rot_index", "too_many_atoms",
                                  "too_many_rot", "self_bond", "not_finite", "disconnected_rot",
                                  "zero_length_axis"])
def test_invalid_ligands_are_rejected(B, case):
    lig = chain(6, rot=[2])
    channels = 2
    if case == "ring":
        lig = Lig(np.arange(12.0).reshape(4, 3), np.zeros(4), [[0, 1], [1, 2], [2, 0], [2, 3]], [0])
    elif case == "type":
        lig.types[3] = 2
    elif case == "bond_index":
        lig.bonds[2, 1] = 6
    elif case == "rot_index":
        lig.rot = np.array([5], np.int32)
    elif case == "too_many_atoms":
        lig = chain(129)
    elif case == "too_many_rot":
        lig = chain(40, rot=list(range(1, 35)))
    elif case == "self_bond":
        lig.bonds[1] = [2, 2]
    elif case == "not_finite":
        lig.xyz[1, 2] = np.nan
    elif case == "zero_length_axis":
        lig.xyz[3] = lig.xyz[2]
    elif case == "disconnected_rot":
        lig = Lig(np.arange(15.0).reshape(5, 3), np.zeros(5), [[0, 1], [2, 3], [3, 4]], [2])
    with pytest.raises(B.ExsError) as ei:
        B.exs_pack_topology(lig, channels)
    assert ei.value.code == B.EXS_EINVAL


@pytest.mark.parametrize("storage,bad,good", [
    (2, 65520.0, 65519.996),          # FP16: 65520 is the tie above 65504 and rounds to inf
    (1, float(np.uint32(0x7f7f8000).view(np.float32)),   # BF16: the tie above the largest
     float(np.uint32(0x7f7f7fff).view(np.float32))),     # finite BF16 rounds to inf
])
def test_texels_that_overflow_16bit_storage_are_refused(B, storage, bad, good):
    """A finite FP32 texel that rounds (to nearest even) to infinity in the requested 16-bit
    storage is refused with EXS_EINVAL before any device work; numpy's own rounding of the same
    values confirms the thresholds (FP16), and a value just below passes validation."""
    if storage == 2:
        assert np.isinf(np.float16(np.float32(bad))) and np.isfinite(np.float16(np.float32(good)))
    vals = np.zeros((1, 2, 2, 2), np.float32)
    vals[0, 1, 1, 1] = bad
    with pytest.raises(B.ExsError) as ei:
        B.exs_load_pocket_grid(vals, 0.5, np.zeros(3), storage)
    assert ei.value.code == B.EXS_EINVAL and "overflows" in str(ei.value)
    vals[0, 1, 1, 1] = -bad
    with pytest.raises(B.ExsError) as ei:
        B.exs_load_pocket_grid(vals, 0.5, np.zeros(3), storage)
    assert ei.value.code == B.EXS_EINVAL
    vals[0, 1, 1, 1] = good
    try:
        pid = B.exs_load_pocket_grid(vals, 0.5, np.zeros(3), storage)
        B.exs_unload_pocket(pid)
    except B.ExsError as e:            # no GPU here: validation passed, the device call failed
        assert e.code != B.EXS_EINVAL, str(e)


@pytest.mark.parametrize("nx,ny,nz,ok", [
    (4096, 2048, 2, False),           # nx * ny = 2^23
    (2, 2, 1 << 23, False),           # nz = 2^23
    (2896, 2896, 2, True),            # nx * ny just below 2^23
])
def test_grid_dimensions_beyond_24_bit_offsets_are_refused(B, nx, ny, nz, ok):
    """The search forms cell offsets with 24-bit multiplies, so a grid whose x-y slice or z edge
    reaches 2^23 texels is refused with EXS_EINVAL before any device work; one just below
    passes validation (here, with no GPU, it then fails on the device call instead)."""
    vals = np.zeros((1, nz, ny, nx), np.float32)
    try:
        pid = B.exs_load_pocket_grid(vals, 0.5, np.zeros(3), B.EXS_F32)
        B.exs_unload_pocket(pid)
        assert ok
    except B.ExsError as e:
        assert (e.code == B.EXS_EINVAL) == (not ok), str(e)
        if not ok:
            assert "2^23" in str(e)
