"""FP64 CPU oracle of the docking search (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It loads ``libexs_oracle.so`` built from
``exs_oracle.c`` (plain C99, FP64, ``-ffp-contract=off``) and shares no code
with the HIP path.  Every function follows a passage of the paper's
Sec. 3.1 ("The dock and score algorithm") with the synthetic score described
in ``exs_oracle.c``.

Inputs are duck-typed: a pocket has ``values`` (float32 [C][N][N][N]),
``spacing`` and ``origin``; a ligand has ``xyz`` (float32 [n,3]), ``types``
(uint8 [n]), ``bonds`` (int32 [nb,2]) and ``rot`` (int32 [B]).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libexs_oracle.so")

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int)
_up = C.POINTER(C.c_ubyte)


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("channels", C.c_int),
                ("h", C.c_double), ("origin", C.c_double * 3), ("values", _fp)]


class _Params(C.Structure):
    _fields_ = [("n_orient", C.c_int), ("torsion_steps", C.c_int), ("passes", C.c_int),
                ("n_offsets", C.c_int), ("offset_step", C.c_double),
                ("clash_cutoff", C.c_double), ("clash_penalty", C.c_double),
                ("near_rel", C.c_double), ("amb_delta", C.c_double)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.orc_grid_value.restype = C.c_double
        L.orc_grid_value.argtypes = [C.POINTER(_Grid), C.c_int, _dp]
        L.orc_bond_distances.argtypes = [C.c_int, C.c_int, _ip, _ip]
        L.orc_moving_set.argtypes = [C.c_int, C.c_int, _ip, C.c_int, _ip, _ip, _up]
        L.orc_rot_topology.argtypes = [C.c_int, C.c_int, _ip, C.c_int, _ip, _ip, _ip, _up]
        L.orc_orientation.argtypes = [C.c_int, C.c_int, _dp]
        L.orc_rotate_about_bond.argtypes = [C.c_int, _dp, C.c_int, C.c_int, _up, C.c_double]
        L.orc_score.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.c_int, _dp, _up,
                                C.c_int, _ip, _dp, _ip, _ip]
        L.orc_pose_from_desc.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.c_int, _fp, _fp,
                                         _fp, _up, C.c_int, _ip, C.c_int, _ip, C.c_int, _ip, _ip,
                                         _dp]
        L.orc_dock_ligand.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.c_int, _fp, _fp, _fp,
                                      _up, C.c_int, _ip, C.c_int, _ip,
                                      _dp, _ip, _ip, _ip, _dp, _dp, _dp, _ip, _ip, _dp, _dp,
                                      C.c_int, _ip, _dp]
        L.orc_dock_batch.argtypes = [C.POINTER(_Grid), C.c_int, C.POINTER(_Params), C.c_int,
                                     _ip, _fp, _fp, _fp, _up, _ip, _ip, _ip, _ip, _ip,
                                     _ip, _dp, _dp, _ip, _ip, _ip, C.c_int]
        L.orc_distance_sum.restype = C.c_double
        L.orc_distance_sum.argtypes = [C.c_int, _dp]
        L.orc_unfold_ligand.argtypes = [C.c_int, _fp, _fp, _fp, C.c_int, _ip, C.c_int, _ip,
                                        C.c_int, C.c_int, C.c_double, _dp, _ip, _ip]
        L.orc_rmsd.restype = C.c_double
        L.orc_rmsd.argtypes = [C.c_int, _dp, _dp]
        L.orc_rank_poses.argtypes = [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double,
                                     C.c_double, _ip, _ip, _ip, _ip]
        L.orc_decision_margin.argtypes = [C.c_int, _dp, _ip, C.c_int, C.c_double, C.c_double,
                                          _dp, _ip]
        L.orc_rescore2.argtypes = [C.POINTER(_Grid), C.c_int, _dp, _up, C.c_int, _ip, C.c_int, _ip,
                                   C.c_double, C.c_double, C.c_double, _dp, _dp]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray], t):
    if a is None:
        return C.cast(None, t)
    return a.ctypes.data_as(t)


@dataclasses.dataclass
class Params:
    n_orient: int
    torsion_steps: int
    passes: int
    n_offsets: int
    offset_step: float = 0.5
    clash_cutoff: float = 2.0
    clash_penalty: float = 1.0
    near_rel: float = 1e-4
    amb_delta: float = 1e-4

    @classmethod
    def of(cls, search, **kw) -> "Params":
        d = dict(n_orient=search.n_orient, torsion_steps=search.torsion_steps,
                 passes=search.passes, n_offsets=search.n_offsets,
                 offset_step=search.offset_step, clash_cutoff=search.clash_cutoff,
                 clash_penalty=search.clash_penalty)
        d.update(kw)
        return cls(**d)

    def c(self) -> _Params:
        return _Params(self.n_orient, self.torsion_steps, self.passes, self.n_offsets,
                       self.offset_step, self.clash_cutoff, self.clash_penalty, self.near_rel,
                       self.amb_delta)


class Grid:
    """A pocket grid held for the oracle (keeps the float32 values alive)."""

    def __init__(self, values: np.ndarray, spacing: float, origin: Sequence[float]):
        self.values = np.ascontiguousarray(values, dtype=np.float32)
        c, nz, ny, nx = self.values.shape
        self.c = _Grid(nx, ny, nz, c, float(spacing), (C.c_double * 3)(*[float(o) for o in origin]),
                       self.values.ctypes.data_as(_fp))

    @classmethod
    def of(cls, pocket) -> "Grid":
        return cls(pocket.values, pocket.spacing, pocket.origin)


def _lig_arrays(lig):
    xyz = np.ascontiguousarray(lig.xyz, dtype=np.float32)
    x = np.ascontiguousarray(xyz[:, 0]); y = np.ascontiguousarray(xyz[:, 1])
    z = np.ascontiguousarray(xyz[:, 2])
    t = np.ascontiguousarray(lig.types, dtype=np.uint8)
    b = np.ascontiguousarray(lig.bonds, dtype=np.int32).reshape(-1)
    r = np.ascontiguousarray(lig.rot, dtype=np.int32)
    return x, y, z, t, b, r


def _check(rc: int):
    if rc != 0:
        raise ValueError("oracle error %d" % rc)


# --- single pieces ----------------------------------------------------------------------------

def grid_value(grid: Grid, channel: int, p: Sequence[float]) -> float:
    pp = np.asarray(p, dtype=np.float64)
    return float(lib().orc_grid_value(C.byref(grid.c), int(channel), _ptr(pp, _dp)))


def bond_distances(n: int, bonds: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1)
    d = np.zeros((n, n), dtype=np.int32)
    _check(lib().orc_bond_distances(n, b.size // 2, _ptr(b, _ip), _ptr(d, _ip)))
    return d


def rot_topology(n: int, bonds: np.ndarray, rot: np.ndarray):
    """(u, v, moving[B, n]) of every rotatable bond."""
    b = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1)
    r = np.ascontiguousarray(rot, dtype=np.int32)
    u = np.zeros(r.size, np.int32); v = np.zeros(r.size, np.int32)
    m = np.zeros((r.size, n), np.uint8)
    _check(lib().orc_rot_topology(n, b.size // 2, _ptr(b, _ip), r.size, _ptr(r, _ip),
                                  _ptr(u, _ip), _ptr(v, _ip), _ptr(m, _up)))
    return u, v, m.astype(bool)


def orientation(k: int, K: int) -> np.ndarray:
    R = np.zeros(9)
    lib().orc_orientation(int(k), int(K), _ptr(R, _dp))
    return R.reshape(3, 3)


def rotate_about_bond(X: np.ndarray, u: int, v: int, moving: np.ndarray, alpha: float) -> np.ndarray:
    Y = np.ascontiguousarray(X, dtype=np.float64).copy()
    m = np.ascontiguousarray(moving, dtype=np.uint8)
    lib().orc_rotate_about_bond(Y.shape[0], _ptr(Y, _dp), int(u), int(v), _ptr(m, _up), float(alpha))
    return Y


def score(grid: Grid, params: Params, X: np.ndarray, types: np.ndarray, bonds: np.ndarray):
    """(E, clashes, ambiguous) of the conformation X as given."""
    Xd = np.ascontiguousarray(X, dtype=np.float64)
    t = np.ascontiguousarray(types, dtype=np.uint8)
    b = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1)
    e = C.c_double(); cl = C.c_int(); am = C.c_int()
    p = params.c()
    _check(lib().orc_score(C.byref(grid.c), C.byref(p), Xd.shape[0], _ptr(Xd, _dp), _ptr(t, _up),
                           b.size // 2, _ptr(b, _ip), C.byref(e), C.byref(cl), C.byref(am)))
    return e.value, cl.value, am.value


def pose_from_desc(grid: Grid, params: Params, lig, k: int, theta: Sequence[int],
                   tau: Sequence[int]) -> np.ndarray:
    x, y, z, t, b, r = _lig_arrays(lig)
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.int64) % params.torsion_steps, dtype=np.int32)
    ta = np.ascontiguousarray(tau, dtype=np.int32)
    X = np.zeros((x.size, 3))
    p = params.c()
    _check(lib().orc_pose_from_desc(C.byref(grid.c), C.byref(p), x.size, _ptr(x, _fp), _ptr(y, _fp),
                                    _ptr(z, _fp), _ptr(t, _up), b.size // 2, _ptr(b, _ip), r.size,
                                    _ptr(r, _ip), int(k), _ptr(th, _ip), _ptr(ta, _ip),
                                    _ptr(X, _dp)))
    return X


def rescore_desc(grid: Grid, params: Params, lig, k: int, theta, tau):
    """(E, clashes, ambiguous, X) of the pose a descriptor stands for."""
    X = pose_from_desc(grid, params, lig, k, theta, tau)
    e, cl, am = score(grid, params, X, lig.types, lig.bonds)
    return e, cl, am, X


# --- whole search -----------------------------------------------------------------------------

def dock_ligand(grid: Grid, params: Params, lig, coords: bool = False, trace_cap: int = 0) -> dict:
    x, y, z, t, b, r = _lig_arrays(lig)
    K, n, B = params.n_orient, x.size, r.size
    out = dict(score=np.zeros(K), clashes=np.zeros(K, np.int32), ambiguous=np.zeros(K, np.int32),
               near_tie=np.zeros(K, np.int32), min_gap=np.zeros(K), min_cand=np.zeros(K),
               start=np.zeros(K), theta=np.zeros((K, B), np.int32), tau=np.zeros((K, 3), np.int32))
    out["coords"] = np.zeros((K, n, 3)) if coords else None
    out["trace"] = np.zeros((K, trace_cap)) if trace_cap else None
    bk = C.c_int(); bs = C.c_double()
    p = params.c()
    _check(lib().orc_dock_ligand(
        C.byref(grid.c), C.byref(p), n, _ptr(x, _fp), _ptr(y, _fp), _ptr(z, _fp), _ptr(t, _up),
        b.size // 2, _ptr(b, _ip), B, _ptr(r, _ip), _ptr(out["score"], _dp),
        _ptr(out["clashes"], _ip), _ptr(out["ambiguous"], _ip), _ptr(out["near_tie"], _ip),
        _ptr(out["min_gap"], _dp), _ptr(out["min_cand"], _dp), _ptr(out["start"], _dp),
        _ptr(out["theta"], _ip), _ptr(out["tau"], _ip), _ptr(out["coords"], _dp),
        _ptr(out["trace"], _dp), int(trace_cap), C.byref(bk), C.byref(bs)))
    out["best_k"] = bk.value
    out["best_score"] = bs.value
    out["near_tie"] = out["near_tie"].astype(bool)
    return out


def distance_sum(X: np.ndarray) -> float:
    """Sum of the distances between all atom pairs of a pose [n,3] (Sec. 3.1, first step)."""
    X = np.ascontiguousarray(X, np.float64)
    return float(lib().orc_distance_sum(X.shape[0], _ptr(X, _dp)))


UNFOLD_PAIR_TOL = 5e-5   # A per changed distance: the near-tie band of an unfolding decision


def unfold_band(n: int, n_moving: int, tol: float = UNFOLD_PAIR_TOL) -> float:
    """Near-tie band of one unfolding decision: a turn changes the n_moving * (n - n_moving)
    distances between turning and fixed atoms, each allowed `tol` in another precision."""
    return tol * n_moving * (n - n_moving)


def unfold_ligand(lig, torsion_steps: int, passes: int, tol: float = UNFOLD_PAIR_TOL) -> dict:
    """Sec. 3.1, first step: turn the rotatable bonds (side without atom 0, S turns each, bonds
    in list order, `passes` passes) to maximise the sum of interatomic distances.  Returns
    xyz [n,3] (FP64, input frame), turns [passes, nrot] and the near-tie count (decisions where
    another turn's sum is within unfold_band of the kept one)."""
    x, y, z, t, b, r = _lig_arrays(lig)
    n, nr = x.size, r.size
    X = np.zeros((n, 3))
    turns = np.zeros((max(passes, 0), nr), np.int32)
    nt = C.c_int()
    _check(lib().orc_unfold_ligand(n, _ptr(x, _fp), _ptr(y, _fp), _ptr(z, _fp), b.size // 2,
                                   _ptr(b, _ip), nr, _ptr(r, _ip), int(torsion_steps), int(passes),
                                   float(tol), _ptr(X, _dp), _ptr(turns, _ip), C.byref(nt)))
    return dict(xyz=X, turns=turns, near_ties=int(nt.value))


def decision_margin(scores: Sequence[float], chosen: int, ambiguous: Optional[Sequence[int]] = None,
                    near_rel: float = 1e-4, clash_penalty: float = 1.0):
    """Near-tie bookkeeping of one greedy decision (Sec. 3.1: the search keeps the best
    candidate): (near_tie, min_gap) for candidate scores with their ambiguous clash-pair
    counts, `chosen` the kept candidate."""
    e = np.ascontiguousarray(scores, np.float64)
    a = None if ambiguous is None else np.ascontiguousarray(ambiguous, np.int32)
    mg = C.c_double()
    nt = C.c_int()
    _check(lib().orc_decision_margin(e.size, _ptr(e, _dp), _ptr(a, _ip), int(chosen),
                                     float(near_rel), float(clash_penalty), C.byref(mg),
                                     C.byref(nt)))
    return bool(nt.value), float(mg.value)


def rmsd(a: np.ndarray, b: np.ndarray) -> float:
    """RMSD of two poses [n,3] of one ligand, same frame (Sec. 3.1, third step)."""
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    return float(lib().orc_rmsd(a.shape[0], _ptr(a, _dp), _ptr(b, _dp)))


def rank_poses(poses: np.ndarray, scores: np.ndarray, thr: float = 3.0, delta: float = 1e-4,
               tol: float = 1e-4) -> dict:
    """Sec. 3.1, third step: cluster the K poses [K,n,3] with the RMSD threshold (greedy
    leaders in score order) and list the leaders by score, then the rest by score.  Returns
    order [K], leader [K] (bool), n_leaders, and the ambiguity counts (RMSD within delta of
    thr; adjacent scores closer than tol * max(|s|, 1))."""
    poses = np.ascontiguousarray(poses, np.float64)
    scores = np.ascontiguousarray(scores, np.float64)
    K, n = poses.shape[0], poses.shape[1]
    order = np.zeros(K, np.int32)
    leader = np.zeros(K, np.int32)
    ar, asc = C.c_int(), C.c_int()
    nl = lib().orc_rank_poses(K, n, _ptr(poses, _dp), _ptr(scores, _dp), float(thr), float(delta),
                              float(tol), _ptr(order, _ip), _ptr(leader, _ip), C.byref(ar),
                              C.byref(asc))
    if nl < 0:
        _check(nl)
    return dict(order=order, leader=leader.astype(bool), n_leaders=int(nl),
                amb_rmsd=int(ar.value), amb_score=int(asc.value))


def dock_batch(grids: Sequence[Grid], params: Params, batch, threads: Optional[int] = None,
               per_orientation: bool = False) -> dict:
    """Dock a CSR batch (OpenMP over ligands).  Returns best_k/best_score per ligand."""
    L = batch.n_ligands
    K = params.n_orient
    arr = (_Grid * len(grids))(*[g.c for g in grids])
    if threads is None:
        threads = os.cpu_count() or 1
    bk = np.zeros(L, np.int32); bs = np.zeros(L)
    sc = np.zeros(L * K) if per_orientation else None
    nt = np.zeros(L * K, np.int32) if per_orientation else None
    th = np.zeros(int(batch.rot_offset[-1]) * K, np.int32) if per_orientation else None
    ta = np.zeros(L * K * 3, np.int32) if per_orientation else None
    p = params.c()
    ao = np.ascontiguousarray(batch.atom_offset, np.int32)
    bo = np.ascontiguousarray(batch.bond_offset, np.int32)
    ro = np.ascontiguousarray(batch.rot_offset, np.int32)
    _check(lib().orc_dock_batch(
        arr, len(grids), C.byref(p), L, _ptr(ao, _ip), _ptr(batch.x, _fp), _ptr(batch.y, _fp),
        _ptr(batch.z, _fp), _ptr(batch.type, _up), _ptr(bo, _ip), _ptr(batch.bond_ij, _ip),
        _ptr(ro, _ip), _ptr(batch.rot_bond, _ip), _ptr(batch.pocket_id, _ip), _ptr(bk, _ip),
        _ptr(bs, _dp), _ptr(sc, _dp), _ptr(nt, _ip), _ptr(th, _ip), _ptr(ta, _ip), int(threads)))
    out = dict(best_k=bk, best_score=bs)
    if per_orientation:
        out.update(score=sc.reshape(L, K), near_tie=nt.reshape(L, K).astype(bool), theta=th,
                   tau=ta.reshape(L, K, 3))
    return out


# --- fourth step: second-stage rescoring ------------------------------------------------------

RESCORE2_EPS = 0.25     # contact-term well depth of the stand-in score
RESCORE2_W = 0.5        # threefold torsion-term weight of the stand-in score


def rescore2(grid: Grid, lig, X: np.ndarray, sigma: float = 2.0, eps: float = RESCORE2_EPS,
             w: float = RESCORE2_W):
    """Sec. 3.1, fourth step: the stand-in chemical score E2 of a pose X [n,3] (grid term +
    smooth contact term over pairs four or more bonds apart + threefold torsion term of the
    rotatable bonds; the definition is in exs_oracle.c).  Returns (E2, (grid, contact,
    torsion))."""
    Xd = np.ascontiguousarray(X, dtype=np.float64)
    t = np.ascontiguousarray(lig.types, dtype=np.uint8)
    b = np.ascontiguousarray(lig.bonds, dtype=np.int32).reshape(-1)
    r = np.ascontiguousarray(lig.rot, dtype=np.int32)
    e = C.c_double()
    parts = np.zeros(3)
    _check(lib().orc_rescore2(C.byref(grid.c), Xd.shape[0], _ptr(Xd, _dp), _ptr(t, _up),
                              b.size // 2, _ptr(b, _ip), r.size, _ptr(r, _ip), float(sigma),
                              float(eps), float(w), C.byref(e), _ptr(parts, _dp)))
    return e.value, tuple(parts.tolist())


def stage2_best(e2: Sequence[float]) -> int:
    """Index of the lowest second-stage score in a ranked list (ties: the earlier entry)."""
    e2 = list(e2)
    j = 0
    for i in range(1, len(e2)):
        if e2[i] < e2[j]:
            j = i
    return j
