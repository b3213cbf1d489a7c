"""Thin ctypes binding of libexs.so: argument marshalling only.

Every function has the name of the C entry point it calls (include/exs.h) and
raises ``ExsError`` on a negative status.  Nothing here computes any part of
the docking search: without the built library the import of ``lib()`` fails
loudly (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; EXS_LIBRARY names another build of the same sources (e.g. one compiled with
# other tuning constants) to load instead
LIB_PATH = os.environ.get("EXS_LIBRARY") or os.path.join(_HERE, "libexs.so")

EXS_OK, EXS_EINVAL, EXS_ENOMEM, EXS_EDEVICE, EXS_ENOTREADY, EXS_ENOENT = 0, -1, -2, -3, -4, -5
EXS_F32, EXS_BF16, EXS_F16 = 0, 1, 2
EXS_FLAG_PERSISTENT, EXS_FLAG_GRAPH, EXS_FLAG_RESCORE2 = 1, 2, 4
EXS_RESCORE2_CONTACT_EPS, EXS_RESCORE2_TORSION_W = 0.25, 0.5
EXS_MAX_ATOMS, EXS_MAX_ROT, EXS_MAX_CHANNELS, EXS_MAX_ORIENT, EXS_MAX_TOPK = 128, 32, 16, 1024, 32

STORAGE = {"f32": EXS_F32, "bf16": EXS_BF16, "f16": EXS_F16}

# exported symbols (kept in step with include/exs.h)
SYMBOLS = ("exs_version", "exs_last_error", "exs_load_pocket_grid", "exs_unload_pocket",
           "exs_upload_ligands", "exs_release_ligands", "exs_pack_topology", "exs_dock_batch", "exs_get_best_poses",
           "exs_get_orientation_results", "exs_get_ranked_poses", "exs_unfold_ligands",
           "exs_get_ligand_coords", "exs_job_elapsed_ms", "exs_job_stage_ms",
           "exs_release_job", "exs_gather_probe",
           "exs_server_create", "exs_server_submit", "exs_server_poll", "exs_server_get_stats",
           "exs_server_destroy", "exs_dock_batch_noalloc", "exs_get_rescored_poses",
           "exs_campaign_run")


class ExsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("exs error %d: %s" % (code, msg))
        self.code = code


class exs_ligand_batch(C.Structure):
    _fields_ = [("n_ligands", C.c_int32), ("atom_offset", C.c_void_p), ("x", C.c_void_p),
                ("y", C.c_void_p), ("z", C.c_void_p), ("type", C.c_void_p),
                ("bond_offset", C.c_void_p), ("bond_ij", C.c_void_p), ("rot_offset", C.c_void_p),
                ("rot_bond", C.c_void_p), ("pocket_id", C.c_void_p)]


class exs_search_params(C.Structure):
    _fields_ = [("n_orient", C.c_int32), ("torsion_steps", C.c_int32), ("passes", C.c_int32),
                ("n_offsets", C.c_int32), ("offset_step_A", C.c_float),
                ("clash_cutoff_A", C.c_float), ("clash_penalty", C.c_float),
                ("top_k", C.c_int32), ("poses_per_lane", C.c_int32),
                ("ligands_per_wg", C.c_int32), ("flags", C.c_int32),
                ("cluster_rmsd_A", C.c_float), ("rank_keep", C.c_int32)]


class exs_server_config(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_iter_ligands", C.c_int32),
                ("max_inflight_iters", C.c_int32), ("max_arena_ligands", C.c_int32),
                ("pad", C.c_int32)]


class exs_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("queued", C.c_int64),
                ("inflight", C.c_int64), ("iterations", C.c_int64), ("ligands_docked", C.c_int64),
                ("arena_ligands", C.c_int64), ("arena_atoms", C.c_int64), ("busy_ms", C.c_double),
                ("budget_bytes", C.c_int64), ("arena_budget_bytes", C.c_int64),
                ("admitted_bytes", C.c_int64), ("peak_admitted_bytes", C.c_int64),
                ("peak_queued", C.c_int64)]


class exs_campaign_config(C.Structure):
    _fields_ = [("chunk_ligands", C.c_int32), ("packers", C.c_int32), ("hit_fraction", C.c_double),
                ("server", exs_server_config)]


class exs_campaign_stats(C.Structure):
    _fields_ = [("ligands", C.c_int64), ("chunks", C.c_int64), ("iterations", C.c_int64),
                ("hits", C.c_int32), ("pad", C.c_int32), ("seconds", C.c_double),
                ("prepass_seconds", C.c_double), ("first_submit_seconds", C.c_double)]


# numpy view of exs_pose_desc (56 bytes, natural alignment)
POSE_DESC = np.dtype([("score", "<f4"), ("pad0", "<f4"), ("score_fp64", "<f8"),
                      ("orient", "<i4"), ("tau", "i1", (3,)), ("n_rot", "u1"),
                      ("theta", "u1", (EXS_MAX_ROT,))])
assert POSE_DESC.itemsize == 56

_lib = None


def lib():
    """Load libexs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libexs.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.exs_version.restype = C.c_char_p
        L.exs_last_error.restype = C.c_char_p
        L.exs_load_pocket_grid.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                           vp, C.c_int, C.c_int, vp, C.POINTER(i32)]
        L.exs_unload_pocket.argtypes = [i32]
        L.exs_upload_ligands.argtypes = [C.POINTER(exs_ligand_batch), vp, C.POINTER(i64)]
        L.exs_release_ligands.argtypes = [i64]
        L.exs_pack_topology.argtypes = [C.c_int, vp, vp, vp, vp, C.c_int, C.c_int, vp, C.c_int,
                                        vp, vp, vp, vp]
        L.exs_dock_batch.argtypes = [i64, C.POINTER(exs_search_params), vp, C.POINTER(i64)]
        L.exs_get_best_poses.argtypes = [i64, C.c_int, vp, vp, vp, vp]
        L.exs_dock_batch_noalloc.argtypes = [i64, C.POINTER(exs_search_params), vp, vp, vp, vp,
                                             vp, vp]
        L.exs_get_orientation_results.argtypes = [i64, vp, vp]
        L.exs_job_elapsed_ms.argtypes = [i64, C.POINTER(C.c_float)]
        L.exs_job_stage_ms.argtypes = [i64, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                       C.POINTER(C.c_float)]
        L.exs_release_job.argtypes = [i64]
        L.exs_get_ranked_poses.argtypes = [i64, C.c_int, vp, vp]
        L.exs_get_rescored_poses.argtypes = [i64, C.c_int, vp, vp, vp]
        L.exs_unfold_ligands.argtypes = [i64, C.c_int, C.c_int, vp, vp]
        L.exs_get_ligand_coords.argtypes = [i64, vp]
        L.exs_gather_probe.argtypes = [i32, i64, C.c_int, C.c_int, C.c_float, C.c_float, C.c_uint32, vp,
                                       C.POINTER(C.c_float), C.POINTER(C.c_double)]
        L.exs_server_create.argtypes = [vp, C.c_int, C.POINTER(exs_search_params),
                                        C.POINTER(exs_server_config), C.POINTER(i64)]
        L.exs_server_submit.argtypes = [i64, C.POINTER(exs_ligand_batch), C.POINTER(i64)]
        L.exs_server_poll.argtypes = [i64, i64, C.c_int, vp, vp, vp, C.POINTER(C.c_double)]
        L.exs_server_get_stats.argtypes = [i64, C.POINTER(exs_server_stats)]
        L.exs_server_destroy.argtypes = [i64]
        L.exs_campaign_run.argtypes = [vp, C.c_int, C.POINTER(exs_search_params),
                                       C.POINTER(exs_ligand_batch), C.POINTER(exs_campaign_config),
                                       vp, vp, C.POINTER(C.c_int32), C.POINTER(exs_campaign_stats)]
        for name in SYMBOLS:
            getattr(L, name).restype = getattr(L, name).restype or C.c_int
        L.exs_version.restype = C.c_char_p
        L.exs_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != EXS_OK:
        raise ExsError(rc, lib().exs_last_error().decode())


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def exs_version() -> str:
    return lib().exs_version().decode()


def exs_load_pocket_grid(values, spacing: float, origin, storage: int = EXS_F32,
                         stream=None) -> int:
    """values: float32 [C][nz][ny][nx] numpy array (host) or torch tensor on the GPU."""
    org = np.ascontiguousarray(origin, dtype=np.float64)
    pid = C.c_int32()
    if hasattr(values, "is_cuda") and values.is_cuda:
        v = values.contiguous()
        c, nz, ny, nx = v.shape
        _check(lib().exs_load_pocket_grid(C.c_void_p(v.data_ptr()), nx, ny, nz, c, float(spacing),
                                          _p(org), int(storage), 1, _stream(stream), C.byref(pid)))
    else:
        v = np.ascontiguousarray(values, dtype=np.float32)
        c, nz, ny, nx = v.shape
        _check(lib().exs_load_pocket_grid(_p(v), nx, ny, nz, c, float(spacing), _p(org),
                                          int(storage), 0, _stream(stream), C.byref(pid)))
    return pid.value


def exs_unload_pocket(pocket_id: int):
    _check(lib().exs_unload_pocket(int(pocket_id)))


def _batch_struct(batch, pocket_ids=None):
    """CSR arrays -> (exs_ligand_batch, keep-alive arrays)."""
    arr = lambda a, t: np.ascontiguousarray(a, dtype=t)
    ao = arr(batch.atom_offset, np.int32)
    x, y, z = arr(batch.x, np.float32), arr(batch.y, np.float32), arr(batch.z, np.float32)
    ty = arr(batch.type, np.uint8)
    bo, bij = arr(batch.bond_offset, np.int32), arr(batch.bond_ij, np.int32)
    ro, rb = arr(batch.rot_offset, np.int32), arr(batch.rot_bond, np.int32)
    pk = np.asarray(batch.pocket_id, dtype=np.int64)
    if pocket_ids is not None:
        pk = np.asarray(pocket_ids, dtype=np.int64)[pk]
    pk = arr(pk, np.int32)
    keep = (ao, x, y, z, ty, bo, bij, ro, rb, pk)
    s = exs_ligand_batch(int(ao.shape[0] - 1), _p(ao), _p(x), _p(y), _p(z), _p(ty), _p(bo),
                         _p(bij), _p(ro), _p(rb), _p(pk))
    return s, keep


def exs_upload_ligands(batch, pocket_ids=None, stream=None) -> int:
    """batch: CSR arrays (attributes atom_offset, x, y, z, type, bond_offset, bond_ij,
    rot_offset, rot_bond, pocket_id).  pocket_ids, if given, maps batch.pocket_id values
    (pocket indices) to loaded pocket handles."""
    s, keep = _batch_struct(batch, pocket_ids)
    out = C.c_int64()
    _check(lib().exs_upload_ligands(C.byref(s), _stream(stream), C.byref(out)))
    return out.value


def exs_release_ligands(batch_id: int):
    _check(lib().exs_release_ligands(int(batch_id)))


def exs_pack_topology(lig, channels: int) -> dict:
    """Host-only packed topology of one ligand (xyz, types, bonds, rot attributes)."""
    xyz = np.ascontiguousarray(lig.xyz, dtype=np.float32)
    x, y, z = (np.ascontiguousarray(xyz[:, a]) for a in range(3))
    t = np.ascontiguousarray(lig.types, dtype=np.uint8)
    b = np.ascontiguousarray(lig.bonds, dtype=np.int32).reshape(-1)
    r = np.ascontiguousarray(lig.rot, dtype=np.int32)
    n, nr = int(xyz.shape[0]), int(r.size)
    excl = np.zeros((n, 4), np.uint32)
    uv = np.zeros((nr, 2), np.int32)
    mv = np.zeros((nr, 4), np.uint32)
    _check(lib().exs_pack_topology(n, _p(x), _p(y), _p(z), _p(t), int(channels), b.size // 2, _p(b),
                                   nr, _p(r), _p(excl), _p(uv), _p(mv)))

    def rows(words, count):
        bits = np.unpackbits(words.astype("<u4").view(np.uint8).reshape(words.shape[0], -1),
                             axis=1, bitorder="little")
        return bits[:, :count].astype(bool)

    return dict(excl=rows(excl, n), rot_u=uv[:, 0].copy(), rot_v=uv[:, 1].copy(),
                moving=rows(mv, n) if nr else np.zeros((0, n), bool))


def search_params(n_orient: int, torsion_steps: int, passes: int, n_offsets: int,
                  offset_step_A: float = 0.5, clash_cutoff_A: float = 2.0,
                  clash_penalty: float = 1.0, top_k: int = 0, poses_per_lane: int = 0,
                  ligands_per_wg: int = 0, flags: int = 0, cluster_rmsd_A: float = 3.0,
                  rank_keep: int = 0) -> exs_search_params:
    return exs_search_params(n_orient, torsion_steps, passes, n_offsets, offset_step_A,
                             clash_cutoff_A, clash_penalty, top_k, poses_per_lane,
                             ligands_per_wg, flags, cluster_rmsd_A, rank_keep)


def exs_dock_batch(batch_id: int, params: exs_search_params, stream=None) -> int:
    out = C.c_int64()
    _check(lib().exs_dock_batch(int(batch_id), C.byref(params), _stream(stream), C.byref(out)))
    return out.value


def exs_dock_batch_noalloc(batch_id: int, params: exs_search_params, best_score, best_orient,
                           best_tau, best_theta, best_coords, stream=None):
    """Enqueue the search of an uploaded batch without device allocation; results go to the
    caller's device tensors (float32 [L], int32 [L], int32 [L], uint8 [R], float32 [A, 3])."""
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    _check(lib().exs_dock_batch_noalloc(int(batch_id), C.byref(params), _stream(stream),
                                        ptr(best_score), ptr(best_orient), ptr(best_tau),
                                        ptr(best_theta), ptr(best_coords)))


def exs_get_best_poses(job: int, n_ligands: int, n_atoms: int, top_k: int = 0, wait: bool = True,
                       coords: bool = True) -> dict:
    best = np.zeros(n_ligands, np.float32)
    desc = np.zeros(n_ligands, POSE_DESC)
    xyz = np.zeros((n_atoms, 3), np.float32) if coords else None
    tk = np.zeros(n_ligands * top_k, POSE_DESC) if top_k > 0 else None
    _check(lib().exs_get_best_poses(int(job), 1 if wait else 0, _p(best), _p(desc), _p(xyz),
                                    _p(tk)))
    return dict(best_score=best, desc=desc, coords=xyz,
                topk=None if tk is None else tk.reshape(n_ligands, top_k))


def exs_get_orientation_results(job: int, n_ligands: int, n_orient: int) -> dict:
    sc = np.zeros(n_ligands * n_orient, np.float32)
    desc = np.zeros(n_ligands * n_orient, POSE_DESC)
    _check(lib().exs_get_orientation_results(int(job), _p(sc), _p(desc)))
    return dict(score=sc.reshape(n_ligands, n_orient), desc=desc.reshape(n_ligands, n_orient))


def exs_unfold_ligands(batch_id: int, torsion_steps: int, passes: int, n_rot: int = 0,
                       stream=None):
    """Unfold the uploaded batch in place; returns the kept turns [passes, n_rot] when
    n_rot (the batch's rotatable bond count) is given, else None."""
    turns = np.zeros((passes, n_rot), np.int32) if n_rot > 0 and passes > 0 else None
    _check(lib().exs_unfold_ligands(int(batch_id), int(torsion_steps), int(passes), _stream(stream),
                                    _p(turns) if turns is not None else None))
    return turns


def exs_get_ligand_coords(batch_id: int, n_atoms: int) -> np.ndarray:
    xyz = np.zeros((n_atoms, 3), np.float32)
    _check(lib().exs_get_ligand_coords(int(batch_id), _p(xyz)))
    return xyz


def exs_get_ranked_poses(job: int, n_ligands: int, rank_keep: int, wait: bool = True):
    """(n_clusters [L], ranked [L, rank_keep]) of a job run with rank_keep > 0."""
    nc = np.zeros(n_ligands, np.int32)
    rk = np.zeros((n_ligands, rank_keep), np.int32)
    _check(lib().exs_get_ranked_poses(int(job), 1 if wait else 0, _p(nc), _p(rk)))
    return nc, rk


def exs_get_rescored_poses(job: int, n_ligands: int, rank_keep: int, wait: bool = True) -> dict:
    """Second-stage scores [L, rank_keep] of the ranked poses, and per ligand the orientation
    and score of the lowest, of a job run with rank_keep > 0 and EXS_FLAG_RESCORE2."""
    sc = np.zeros((n_ligands, rank_keep), np.float64)
    bk = np.zeros(n_ligands, np.int32)
    bs = np.zeros(n_ligands, np.float64)
    _check(lib().exs_get_rescored_poses(int(job), 1 if wait else 0, _p(sc), _p(bk), _p(bs)))
    return dict(score2=sc, best_orient=bk, best_score2=bs)


def exs_job_elapsed_ms(job: int) -> float:
    ms = C.c_float()
    _check(lib().exs_job_elapsed_ms(int(job), C.byref(ms)))
    return float(ms.value)


def exs_job_stage_ms(job: int) -> dict:
    """Device ms of the search, the ranking and the second-stage rescoring of an eager ranked
    job (-1 for a step not run; an unstaged job gives its whole time as "dock")."""
    d, r, q = C.c_float(), C.c_float(), C.c_float()
    _check(lib().exs_job_stage_ms(int(job), C.byref(d), C.byref(r), C.byref(q)))
    return {"dock": float(d.value), "rank": float(r.value), "rescore2": float(q.value)}


def exs_release_job(job: int):
    _check(lib().exs_release_job(int(job)))


def exs_gather_probe(pocket_id: int, n_lanes: int, lookups_per_lane: int, half_edge_A: float,
                     walk_step_A: float = 0.0, seed: int = 1, batch: int = 16, stream=None):
    """Device time (ms) and checksum of the texel-gather probe on a loaded pocket."""
    ms = C.c_float()
    chk = C.c_double()
    _check(lib().exs_gather_probe(int(pocket_id), int(n_lanes), int(lookups_per_lane), int(batch),
                                  float(half_edge_A), float(walk_step_A), int(seed) & 0xffffffff,
                                  _stream(stream), C.byref(ms), C.byref(chk)))
    return float(ms.value), float(chk.value)


def exs_server_create(pocket_ids, params: exs_search_params, hbm_budget_bytes: int = 0,
                      max_iter_ligands: int = 0, max_inflight_iters: int = 0,
                      max_arena_ligands: int = 0) -> int:
    pk = np.ascontiguousarray(pocket_ids, dtype=np.int32)
    cfg = exs_server_config(int(hbm_budget_bytes), int(max_iter_ligands), int(max_inflight_iters),
                            int(max_arena_ligands), 0)
    out = C.c_int64()
    _check(lib().exs_server_create(_p(pk), int(pk.size), C.byref(params), C.byref(cfg),
                                   C.byref(out)))
    return out.value


def exs_server_submit(server: int, batch, pocket_ids=None) -> int:
    s, keep = _batch_struct(batch, pocket_ids)
    out = C.c_int64()
    _check(lib().exs_server_submit(int(server), C.byref(s), C.byref(out)))
    return out.value


def exs_server_poll(server: int, request: int, n_ligands: int, n_atoms: int, wait: bool = True):
    """Returns None while the request is queued or running (wait=False), else a dict."""
    best = np.zeros(n_ligands, np.float32)
    desc = np.zeros(n_ligands, POSE_DESC)
    xyz = np.zeros((n_atoms, 3), np.float32)
    lat = C.c_double()
    rc = lib().exs_server_poll(int(server), int(request), 1 if wait else 0, _p(best), _p(desc),
                               _p(xyz), C.byref(lat))
    if rc == EXS_ENOTREADY:
        return None
    _check(rc)
    return dict(best_score=best, desc=desc, coords=xyz, latency_ms=lat.value)


def exs_server_get_stats(server: int) -> dict:
    st = exs_server_stats()
    _check(lib().exs_server_get_stats(int(server), C.byref(st)))
    return {name: getattr(st, name) for name, _ in exs_server_stats._fields_}


def exs_server_destroy(server: int):
    _check(lib().exs_server_destroy(int(server)))


def exs_campaign_run(pocket_ids, params: exs_search_params, library, chunk_ligands: int = 0,
                     packers: int = 0, hit_fraction: float = 0.0, hbm_budget_bytes: int = 0,
                     max_iter_ligands: int = 0, max_inflight_iters: int = 0,
                     max_arena_ligands: int = 0, library_pocket_ids=None) -> dict:
    """Screen a host CSR library (pocket_id: handles, or indices into library_pocket_ids).
    Returns best_score [L], hits (library indices, best first) and the campaign stats."""
    pk = np.ascontiguousarray(pocket_ids, dtype=np.int32)
    s, keep = _batch_struct(library, library_pocket_ids)
    L = int(s.n_ligands)
    n_hits_max = max(1, int(round(L * (hit_fraction if hit_fraction > 0 else 0.01))))
    best = np.zeros(L, np.float32)
    hits = np.zeros(n_hits_max + 1, np.int32)
    nh = C.c_int32()
    st = exs_campaign_stats()
    cfg = exs_campaign_config(int(chunk_ligands), int(packers), float(hit_fraction),
                              exs_server_config(int(hbm_budget_bytes), int(max_iter_ligands),
                                                int(max_inflight_iters), int(max_arena_ligands), 0))
    _check(lib().exs_campaign_run(_p(pk), int(pk.size), C.byref(params), C.byref(s), C.byref(cfg),
                                  _p(best), _p(hits), C.byref(nh), C.byref(st)))
    return dict(best_score=best, hits=hits[:nh.value].copy(),
                stats={name: getattr(st, name) for name, _ in exs_campaign_stats._fields_})
