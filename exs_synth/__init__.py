"""Seeded synthetic inputs for the docking hot path.

This module only *draws inputs*: pocket grids, ligand trees and request traces.
It holds none of the docking method's arithmetic (no scoring, no rotation of
torsional bonds, no search), so both the FP64 oracle and the HIP path can take
their inputs from it without sharing any of the method.

Every object comes from its own counter-based stream::

    Generator(PCG64(SeedSequence([SEED, workload_id, kind, index])))

with kind 0 = pocket, 1 = ligand, 2 = request trace.  Any pocket, ligand or
request can therefore be regenerated on its own, which the "alone vs. in the
mix" serving check relies on.

Workloads (sizes follow the synthetic stand-ins for the paper's screening
campaign, Sec. 3.1 "dock and score" and Sec. 4 "experiment"):

* ``small``     -- 1 pocket 48^3 x 4 channels at 0.5 A; 64 ligands of 24 atoms
                   and 4 rotatable bonds; 64 orientations, 16 torsion steps,
                   1 pass, no rigid offsets.
* ``scale``     -- 1 pocket 96^3 x 8 channels at 0.375 A; 10,000 ligands with
                   atoms ~ U{20..60} and rotatable bonds ~ U{0..12}; 256
                   orientations, 32 torsion steps, 2 passes, 27 offsets.
* ``batched``   -- 15 pockets with edges drawn from {64,80,96,112,128} at
                   0.375 A, 8 channels; 100,000 ligands, atoms log-normal
                   (median 35, sigma 0.4 in ln-space, clipped to [10, 90]),
                   rotatable bonds ~ U{0..15}, random pocket each.
* ``precision`` -- the batched inputs (same streams), grids stored 16-bit.
* ``serving``   -- the batched pockets; Poisson request trace, request sizes
                   log-uniform on 1..512 ligands.

Pocket grid: 300 pseudo-atoms uniform in a 10 A ball around the grid centre,
per-channel weights w ~ U(-1, 1); texel value = sum_a w_a exp(-d^2/(2*1.2^2)),
plus 10.0 where any pseudo-atom is closer than 1.2 A.  Node-centred texels:
texel (i, j, k) sits at origin + h*(i, j, k), origin = -h(N-1)/2 per axis, so
the grid centre is (0, 0, 0).  Computed in FP64, stored as round-to-nearest
FP32, layout [channel][z][y][x] with x fastest.

Ligand: a random tree.  Atom 0 at the origin, atom 1 at +1.5 x.  Every later
atom bonds to a uniformly chosen earlier atom of degree < 4 at 1.5 A, with a
109.5 degree bond angle and a uniform dihedral.  Angle reference: the
parent's parent (for the root, atom 1).  Dihedral reference: the lowest-index
neighbour of the angle reference other than the parent, else the fixed point
(angle reference + z), or + y if that is collinear.  Types uniform over the
channels.  Rotatable bonds: a uniform sample (without replacement) of the
non-terminal tree edges, listed in bond order; the requested count is clipped
to the number available.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

SEED = 211011644

KIND_POCKET = 0
KIND_LIGAND = 1
KIND_TRACE = 2

NMAX_DRAW = 128          # fixed draw width per ligand: counter-based regeneration
BOND_LENGTH = 1.5
BOND_ANGLE_DEG = 109.5


@dataclasses.dataclass(frozen=True)
class SearchSettings:
    n_orient: int
    torsion_steps: int
    passes: int
    n_offsets: int
    offset_step: float = 0.5
    clash_cutoff: float = 2.0
    clash_penalty: float = 1.0
    top_k: int = 0


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    wid: int                     # stream id used in the seed sequence
    n_ligands: int
    n_pockets: int
    pocket_edges: Sequence[int]  # one edge (fixed) or the set drawn from
    spacing: float
    channels: int
    atoms: tuple                 # ("fixed", n) | ("uniform", lo, hi) | ("lognormal", median, sigma, lo, hi)
    rot: tuple                   # ("fixed", b) | ("uniform", lo, hi)
    search: SearchSettings
    pocket_wid: Optional[int] = None   # pockets drawn from another workload's streams
    ligand_wid: Optional[int] = None   # ligands drawn from another workload's streams


SMALL = Workload("small", 1, 64, 1, (48,), 0.5, 4, ("fixed", 24), ("fixed", 4),
                 SearchSettings(64, 16, 1, 1))
SCALE = Workload("scale", 2, 10_000, 1, (96,), 0.375, 8, ("uniform", 20, 60), ("uniform", 0, 12),
                 SearchSettings(256, 32, 2, 27))
BATCHED = Workload("batched", 3, 100_000, 15, (64, 80, 96, 112, 128), 0.375, 8,
                   ("lognormal", 35.0, 0.4, 10, 90), ("uniform", 0, 15),
                   SearchSettings(256, 32, 2, 27))
PRECISION = Workload("precision", 4, 100_000, 15, (64, 80, 96, 112, 128), 0.375, 8,
                     ("lognormal", 35.0, 0.4, 10, 90), ("uniform", 0, 15),
                     SearchSettings(256, 32, 2, 27, top_k=8), pocket_wid=3, ligand_wid=3)
SERVING = Workload("serving", 5, 0, 15, (64, 80, 96, 112, 128), 0.375, 8,
                   ("lognormal", 35.0, 0.4, 10, 90), ("uniform", 0, 15),
                   SearchSettings(256, 32, 2, 27), pocket_wid=3)

WORKLOADS: Dict[str, Workload] = {w.name: w for w in (SMALL, SCALE, BATCHED, PRECISION, SERVING)}


def stream(wid: int, kind: int, index: int) -> np.random.Generator:
    """The counter-based generator of one object."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED, wid, kind, index])))


# ----------------------------------------------------------------------------------------------
# Pockets
# ----------------------------------------------------------------------------------------------

@dataclasses.dataclass
class Pocket:
    values: np.ndarray      # float32 [C][N][N][N], x fastest
    spacing: float
    origin: np.ndarray      # float64 [3], position of texel (0,0,0)
    pseudo_xyz: np.ndarray  # float64 [300,3]
    pseudo_w: np.ndarray    # float64 [300,C]

    @property
    def n(self) -> int:
        return self.values.shape[-1]

    @property
    def channels(self) -> int:
        return self.values.shape[0]


def pocket_grid_values(edge: int, spacing: float, pseudo_xyz: np.ndarray, pseudo_w: np.ndarray,
                       sigma: float = 1.2, core_radius: float = 1.2, core_value: float = 10.0
                       ) -> np.ndarray:
    """Texel values of a synthetic pocket, FP64 -> RNE FP32, layout [C][z][y][x].

    The Gaussian sum is evaluated separably (exp(-d^2/2s^2) is the product of the three
    per-axis factors), as one small matrix product per z slice; the +core_value cores are
    marked by exact distance tests in the box around each pseudo-atom."""
    n = int(edge)
    c = pseudo_w.shape[1]
    origin = -spacing * (n - 1) / 2.0
    axis = origin + spacing * np.arange(n, dtype=np.float64)
    two_s2 = 2.0 * sigma * sigma
    gx = np.exp(-(axis[None, :] - pseudo_xyz[:, 0:1]) ** 2 / two_s2)   # [300, n]
    gy = np.exp(-(axis[None, :] - pseudo_xyz[:, 1:2]) ** 2 / two_s2)
    gz = np.exp(-(axis[None, :] - pseudo_xyz[:, 2:3]) ** 2 / two_s2)
    out = np.empty((c, n, n, n), dtype=np.float32)
    wy = pseudo_w[:, :, None] * gy[:, None, :]                           # [300, C, n(y)]
    wy = wy.transpose(1, 2, 0).reshape(c * n, -1)                        # [(C, y), 300]
    for k in range(n):
        m = gx * gz[:, k:k + 1]                                          # [300, n(x)]
        out[:, k, :, :] = (wy @ m).reshape(c, n, n).astype(np.float32)
    # cores: texels closer than core_radius to any pseudo-atom
    core = np.zeros((n, n, n), dtype=bool)
    reach = int(np.ceil(core_radius / spacing)) + 1
    for a in range(pseudo_xyz.shape[0]):
        ctr = np.round((pseudo_xyz[a] - origin) / spacing).astype(int)
        lo = np.maximum(ctr - reach, 0)
        hi = np.minimum(ctr + reach + 1, n)
        if np.any(lo >= hi):
            continue
        zz, yy, xx = np.meshgrid(axis[lo[2]:hi[2]], axis[lo[1]:hi[1]], axis[lo[0]:hi[0]],
                                 indexing="ij")
        d = np.sqrt((xx - pseudo_xyz[a, 0]) ** 2 + (yy - pseudo_xyz[a, 1]) ** 2
                    + (zz - pseudo_xyz[a, 2]) ** 2)
        core[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] |= d < core_radius
    if core.any():
        idx = np.nonzero(core)
        for ch in range(c):
            # add in FP64 before rounding, as the definition states
            vals = (wy.reshape(c, n, -1)[ch][idx[1]] * (gx[:, idx[2]] * gz[:, idx[0]]).T).sum(axis=1)
            out[ch][idx] = (vals + core_value).astype(np.float32)
    return out


def pocket_grid_values_direct(edge: int, spacing: float, pseudo_xyz: np.ndarray,
                              pseudo_w: np.ndarray, sigma: float = 1.2, core_radius: float = 1.2,
                              core_value: float = 10.0) -> np.ndarray:
    """The same texels by the literal formula (slow; used to check the separable form)."""
    n = int(edge)
    c = pseudo_w.shape[1]
    origin = -spacing * (n - 1) / 2.0
    axis = origin + spacing * np.arange(n, dtype=np.float64)
    out = np.empty((c, n, n, n), dtype=np.float32)
    two_s2 = 2.0 * sigma * sigma
    px, py, pz = pseudo_xyz[:, 0], pseudo_xyz[:, 1], pseudo_xyz[:, 2]
    dx2 = (axis[:, None] - px[None, :]) ** 2
    for k in range(n):
        dz2 = (axis[k] - pz) ** 2
        d2 = (dz2[None, None, :] + ((axis[:, None] - py[None, :]) ** 2)[:, None, :]
              + dx2[None, :, :]).reshape(n * n, -1)
        g = np.exp(-d2 / two_s2) @ pseudo_w
        core = np.sqrt(d2.min(axis=1)) < core_radius
        g[core] += core_value
        out[:, k, :, :] = g.T.reshape(c, n, n).astype(np.float32)
    return out


def make_pocket(workload: Workload | str, index: int = 0) -> Pocket:
    wl = WORKLOADS[workload] if isinstance(workload, str) else workload
    wid = wl.pocket_wid if wl.pocket_wid is not None else wl.wid
    rng = stream(wid, KIND_POCKET, index)
    edges = list(wl.pocket_edges)
    edge = int(edges[0]) if len(edges) == 1 else int(rng.choice(np.asarray(edges)))
    u = rng.random(300)
    d = rng.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    xyz = d * (10.0 * np.cbrt(u))[:, None]
    w = rng.uniform(-1.0, 1.0, size=(300, wl.channels))
    vals = pocket_grid_values(edge, wl.spacing, xyz, w)
    org = np.full(3, -wl.spacing * (edge - 1) / 2.0)
    return Pocket(vals, wl.spacing, org, xyz, w)


def make_pockets(workload: Workload | str, indices: Optional[Sequence[int]] = None,
                 threads: int = 8) -> List[Pocket]:
    """make_pocket for several indices (default: every pocket of the workload) on a thread
    pool; the grids are the same as one by one (each pocket draws from its own stream)."""
    from concurrent.futures import ThreadPoolExecutor
    wl = WORKLOADS[workload] if isinstance(workload, str) else workload
    idx = list(range(wl.n_pockets)) if indices is None else list(indices)
    with ThreadPoolExecutor(max(1, min(threads, len(idx)))) as ex:
        return list(ex.map(lambda i: make_pocket(wl, i), idx))


def pocket_edge(workload: Workload | str, index: int = 0) -> int:
    """Edge of a pocket without building its grid (same draw order as make_pocket)."""
    wl = WORKLOADS[workload] if isinstance(workload, str) else workload
    wid = wl.pocket_wid if wl.pocket_wid is not None else wl.wid
    edges = list(wl.pocket_edges)
    if len(edges) == 1:
        return int(edges[0])
    return int(stream(wid, KIND_POCKET, index).choice(np.asarray(edges)))


def to_bf16_rne(values: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 (round to nearest even), returned widened back to float32."""
    b = np.ascontiguousarray(values, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).reshape(values.shape)


def to_f16_rne(values: np.ndarray) -> np.ndarray:
    """FP32 -> FP16 (round to nearest even), returned widened back to float32."""
    return np.asarray(values, dtype=np.float32).astype(np.float16).astype(np.float32)


# ----------------------------------------------------------------------------------------------
# Ligands
# ----------------------------------------------------------------------------------------------

@dataclasses.dataclass
class Ligand:
    xyz: np.ndarray      # float32 [n,3]
    types: np.ndarray    # uint8 [n]
    bonds: np.ndarray    # int32 [nb,2]
    rot: np.ndarray      # int32 [B], indices into bonds
    pocket: int = 0

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


@dataclasses.dataclass
class LigandBatch:
    """CSR form of a list of ligands (the layout the C ABI takes)."""
    atom_offset: np.ndarray   # int32 [L+1]
    x: np.ndarray             # float32 [A]
    y: np.ndarray
    z: np.ndarray
    type: np.ndarray          # uint8 [A]
    bond_offset: np.ndarray   # int32 [L+1]
    bond_ij: np.ndarray       # int32 [2*nb], local atom indices
    rot_offset: np.ndarray    # int32 [L+1]
    rot_bond: np.ndarray      # int32 [R], index into the ligand's own bond list
    pocket_id: np.ndarray     # int32 [L]

    @property
    def n_ligands(self) -> int:
        return int(self.atom_offset.shape[0] - 1)

    def ligand(self, i: int) -> Ligand:
        a0, a1 = int(self.atom_offset[i]), int(self.atom_offset[i + 1])
        b0, b1 = int(self.bond_offset[i]), int(self.bond_offset[i + 1])
        r0, r1 = int(self.rot_offset[i]), int(self.rot_offset[i + 1])
        xyz = np.stack([self.x[a0:a1], self.y[a0:a1], self.z[a0:a1]], axis=1)
        return Ligand(xyz.astype(np.float32), self.type[a0:a1].copy(),
                      self.bond_ij[2 * b0:2 * b1].reshape(-1, 2).copy(),
                      self.rot_bond[r0:r1].copy(), int(self.pocket_id[i]))

    def subset(self, idx: Sequence[int]) -> "LigandBatch":
        return batch_from_ligands([self.ligand(int(i)) for i in idx])


def batch_from_ligands(ligs: List[Ligand]) -> LigandBatch:
    n = np.array([l.n for l in ligs], dtype=np.int64)
    nb = np.array([l.bonds.shape[0] for l in ligs], dtype=np.int64)
    nr = np.array([l.rot.shape[0] for l in ligs], dtype=np.int64)
    ao = np.zeros(len(ligs) + 1, np.int32); ao[1:] = np.cumsum(n)
    bo = np.zeros(len(ligs) + 1, np.int32); bo[1:] = np.cumsum(nb)
    ro = np.zeros(len(ligs) + 1, np.int32); ro[1:] = np.cumsum(nr)
    cat = lambda arrs, dt: (np.concatenate(arrs).astype(dt) if arrs else np.zeros(0, dt))
    xyz = cat([l.xyz for l in ligs], np.float32).reshape(-1, 3) if ligs else np.zeros((0, 3), np.float32)
    return LigandBatch(
        ao, np.ascontiguousarray(xyz[:, 0]), np.ascontiguousarray(xyz[:, 1]),
        np.ascontiguousarray(xyz[:, 2]), cat([l.types for l in ligs], np.uint8),
        bo, cat([l.bonds.reshape(-1) for l in ligs], np.int32), ro,
        cat([l.rot for l in ligs], np.int32),
        np.array([l.pocket for l in ligs], dtype=np.int32))


def _draw_ligand_params(wl: Workload, rng: np.random.Generator):
    kind = wl.atoms[0]
    if kind == "fixed":
        n = int(wl.atoms[1])
    elif kind == "uniform":
        n = int(rng.integers(wl.atoms[1], wl.atoms[2] + 1))
    else:
        _, med, sig, lo, hi = wl.atoms
        n = int(np.clip(np.round(np.exp(rng.normal(math.log(med), sig))), lo, hi))
    if wl.rot[0] == "fixed":
        b = int(wl.rot[1])
    else:
        b = int(rng.integers(wl.rot[1], wl.rot[2] + 1))
    pocket = int(rng.integers(0, wl.n_pockets)) if wl.n_pockets > 1 else 0
    types = rng.integers(0, wl.channels, size=NMAX_DRAW).astype(np.uint8)
    u_parent = rng.random(NMAX_DRAW)
    phi = rng.random(NMAX_DRAW) * (2.0 * math.pi)
    rot_key = rng.random(NMAX_DRAW)
    return n, b, pocket, types, u_parent, phi, rot_key


def _nerf(a, b, c, r, theta, phi):
    """Place D with |CD| = r, angle BCD = theta, dihedral ABCD = phi (vectorised over rows)."""
    bc = c - b
    bc /= np.linalg.norm(bc, axis=-1, keepdims=True)
    nrm = np.cross(b - a, bc)
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    m = np.cross(nrm, bc)
    d0 = -r * math.cos(theta)
    d1 = r * math.sin(theta) * np.cos(phi)
    d2 = r * math.sin(theta) * np.sin(phi)
    return c + d0 * bc + d1[:, None] * m + d2[:, None] * nrm


def _build_trees(n: np.ndarray, breq: np.ndarray, u_parent: np.ndarray, phi: np.ndarray,
                 rot_key: np.ndarray):
    """Vectorised random-tree construction over L ligands (rows)."""
    L = n.shape[0]
    nmax = int(n.max()) if L else 0
    pos = np.zeros((L, max(nmax, 2), 3))
    par = np.full((L, max(nmax, 2)), -1, np.int64)
    deg = np.zeros((L, max(nmax, 2)), np.int64)
    child1 = np.full((L, max(nmax, 2)), -1, np.int64)   # lowest-index child
    child2 = np.full((L, max(nmax, 2)), -1, np.int64)   # second lowest-index child
    rows = np.arange(L)
    theta = math.radians(BOND_ANGLE_DEG)
    zhat = np.array([0.0, 0.0, 1.0]); yhat = np.array([0.0, 1.0, 0.0])

    def add_child(rr, p, ch):
        c1 = child1[rr, p]
        first = c1 < 0
        child1[rr[first], p[first]] = ch[first]
        sec = (~first) & (child2[rr, p] < 0)
        child2[rr[sec], p[sec]] = ch[sec]

    if nmax >= 2:
        act = n > 1
        rr = rows[act]
        pos[rr, 1] = [BOND_LENGTH, 0.0, 0.0]
        par[rr, 1] = 0
        deg[rr, 0] += 1; deg[rr, 1] = 1
        add_child(rr, np.zeros(rr.shape[0], np.int64), np.ones(rr.shape[0], np.int64))
    for a in range(2, nmax):
        act = n > a
        rr = rows[act]
        if rr.size == 0:
            break
        elig = deg[rr, :a] < 4
        cnt = elig.sum(axis=1)
        pick = np.minimum(np.floor(u_parent[rr, a] * cnt).astype(np.int64), cnt - 1)
        csum = np.cumsum(elig, axis=1)
        p = np.argmax(csum > pick[:, None], axis=1)
        # angle reference B
        bref = np.where(p == 0, 1, par[rr, np.maximum(p, 0)])
        bref = np.where(p == 0, 1, bref)
        # dihedral reference A: lowest-index neighbour of B other than p
        parb = np.where(bref == 0, -1, par[rr, bref])
        c1 = child1[rr, bref]; c2 = child2[rr, bref]
        alt = np.where(c1 != p, c1, c2)
        aref = np.where((parb >= 0) & (parb != p), parb, alt)
        pb = pos[rr, bref]; pc = pos[rr, p]
        has_a = aref >= 0
        pa = np.where(has_a[:, None], pos[rr, np.maximum(aref, 0)], pb + zhat[None, :])
        # fall back to +y if the fixed point is collinear with B->C
        cb = pc - pb
        col = (~has_a) & (np.linalg.norm(np.cross(cb, zhat[None, :]), axis=1) < 1e-9)
        pa[col] = pb[col] + yhat[None, :]
        pos[rr, a] = _nerf(pa, pb, pc, BOND_LENGTH, theta, phi[rr, a])
        par[rr, a] = p
        deg[rr, p] += 1; deg[rr, a] = 1
        add_child(rr, p, np.full(rr.shape[0], a, np.int64))
    # rotatable bonds: non-terminal edges (both ends of degree >= 2); bond index = child - 1
    rots = []
    for l in range(L):
        nl = int(n[l])
        child = np.arange(1, nl)
        nonterm = (deg[l, child] >= 2) & (deg[l, par[l, child]] >= 2)
        cand = child[nonterm]
        k = min(int(breq[l]), cand.size)
        order = np.argsort(rot_key[l, cand], kind="stable")[:k]
        rots.append(np.sort(cand[order] - 1).astype(np.int32))
    return pos, par, rots


def make_ligands(workload: Workload | str, start: int, count: int) -> List[Ligand]:
    """Ligands start..start+count-1 of a workload (each from its own stream)."""
    wl = WORKLOADS[workload] if isinstance(workload, str) else workload
    wid = wl.ligand_wid if wl.ligand_wid is not None else wl.wid
    if count <= 0:
        return []
    draws = [_draw_ligand_params(wl, stream(wid, KIND_LIGAND, start + i)) for i in range(count)]
    n = np.array([d[0] for d in draws], np.int64)
    breq = np.array([d[1] for d in draws], np.int64)
    u_parent = np.stack([d[4] for d in draws]); phi = np.stack([d[5] for d in draws])
    rot_key = np.stack([d[6] for d in draws])
    pos, par, rots = _build_trees(n, breq, u_parent, phi, rot_key)
    out = []
    for l, d in enumerate(draws):
        nl = int(n[l])
        bonds = np.stack([par[l, 1:nl], np.arange(1, nl)], axis=1).astype(np.int32)
        out.append(Ligand(pos[l, :nl].astype(np.float32), d[3][:nl].copy(), bonds, rots[l], d[2]))
    return out


def make_ligand_batch(workload: Workload | str, start: int = 0, count: Optional[int] = None,
                      chunk: int = 4096) -> LigandBatch:
    wl = WORKLOADS[workload] if isinstance(workload, str) else workload
    if count is None:
        count = wl.n_ligands - start
    ligs: List[Ligand] = []
    for s in range(start, start + count, chunk):
        ligs.extend(make_ligands(wl, s, min(chunk, start + count - s)))
    return batch_from_ligands(ligs)


# ----------------------------------------------------------------------------------------------
# Request trace (serving)
# ----------------------------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    pocket: int
    ligand_start: int     # ligands ligand_start .. ligand_start+size-1 of the serving stream
    size: int


def make_trace(n_requests: int, rate_per_s: float, n_pockets: int = 15, max_size: int = 512,
               wid: int = 5) -> List[Request]:
    """Poisson arrivals (exponential gaps at ``rate_per_s``); sizes log-uniform on 1..max_size."""
    rng = stream(wid, KIND_TRACE, 0)
    gaps = rng.exponential(1.0, size=n_requests) / rate_per_s
    sizes = np.clip(np.floor(np.exp(rng.uniform(0.0, math.log(max_size + 1), size=n_requests))),
                    1, max_size).astype(np.int64)
    pockets = rng.integers(0, n_pockets, size=n_requests)
    t = np.cumsum(gaps)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    return [Request(i, float(t[i]), int(pockets[i]), int(starts[i]), int(sizes[i]))
            for i in range(n_requests)]


def serving_ligands(req: Request) -> List[Ligand]:
    """The ligands of one request, each regenerated from its own counter-based stream."""
    ligs = make_ligands(SERVING, req.ligand_start, req.size)
    for l in ligs:
        l.pocket = req.pocket
    return ligs
