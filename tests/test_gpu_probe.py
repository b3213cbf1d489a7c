"""The texel-gather probe computes what it claims: the sum, over its lanes, of trilinear
lookups at the points its hash generates.  The points are regenerated here from the hash's
published definition (Wellons' "lowbias32" finalizer) and scored by the FP64 oracle."""
import numpy as np
import pytest

import exs_synth as S

pytestmark = pytest.mark.gpu

M32 = 0xffffffff


def mix32(x):
    x = np.asarray(x, np.uint64) & M32
    x ^= x >> 16
    x = (x * 0x7feb352d) & M32
    x ^= x >> 15
    x = (x * 0x846ca68b) & M32
    x ^= x >> 16
    return x


def probe_points(pocket, n_lanes, per_lane, half_A, seed):
    """Grid-unit points [lanes, per_lane, 3] and channels [lanes, per_lane] of the probe
    (independent-point mode), in the probe's FP32 arithmetic."""
    f32 = np.float32
    inv_h = f32(1.0 / pocket.spacing)
    n = pocket.values.shape[-1]
    centre = pocket.origin + pocket.spacing * (n - 1) / 2.0
    c0 = (centre.astype(f32) - pocket.origin.astype(f32)) * inv_h
    half = f32(f32(half_A) * inv_h)
    unit = f32(2.0 / 1023.0)
    lanes = np.arange(n_lanes, dtype=np.uint64)
    h = mix32(np.uint64(seed) ^ mix32(lanes))
    pts = np.zeros((n_lanes, per_lane, 3), np.float64)
    chans = np.zeros((n_lanes, per_lane), np.int64)
    C = pocket.values.shape[0]
    c = (lanes // 256) % C

    def coords(h):
        out = []
        for a in range(3):
            k = ((h >> np.uint64(10 * a)) & np.uint64(1023)).astype(np.float64)
            v = (k * float(unit) - 1.0).astype(f32)                        # one rounding: fma
            out.append((float(half) * v.astype(np.float64) + float(c0[a])).astype(f32))
        return out

    p = coords(h)
    for i in range(per_lane):
        pts[:, i, :] = np.stack(p, axis=1)
        chans[:, i] = c
        if (i + 1) % 32 == 0:                  # runs of 32 lookups keep one channel
            c = np.where(c + 1 == C, 0, c + 1)
        h = mix32(h + np.uint64(0x9e3779b9))
        p = coords(h)
    return pts, chans


def test_gather_probe_sum_matches_oracle(oracle_lib):
    import torch
    assert torch.cuda.is_available()
    from paper_2110_11644_amd import binding as B
    O = oracle_lib
    pocket = S.make_pocket("small")
    pid = B.exs_load_pocket_grid(pocket.values, pocket.spacing, pocket.origin, B.STORAGE["f32"])
    try:
        n_lanes, per_lane, half, seed = 512, 96, 9.0, 12345
        ms, chk = B.exs_gather_probe(pid, n_lanes, per_lane, half, 0.0, seed)
        assert ms > 0.0
        pts, chans = probe_points(pocket, n_lanes, per_lane, half, seed)
        g = O.Grid.of(pocket)
        ref, ref_abs = 0.0, 0.0
        for l in range(n_lanes):
            for i in range(per_lane):
                x = pocket.origin + pts[l, i] * pocket.spacing
                v = O.grid_value(g, int(chans[l, i]), x)
                ref += v
                ref_abs += abs(v)
        # FP32 lookups and per-lane FP32 sums: a few ulps of each term
        assert abs(chk - ref) <= 1e-5 * ref_abs, (chk, ref, ref_abs)
        # the same points summed in the same order, whatever the number of lookups in flight
        for nb in (8, 32):
            _, c2 = B.exs_gather_probe(pid, n_lanes, per_lane, half, 0.0, seed, batch=nb)
            assert c2 == chk
        # the walk mode runs and stays finite
        ms2, chk2 = B.exs_gather_probe(pid, 1024, 64, 12.0, 0.7, seed)
        assert ms2 > 0.0 and np.isfinite(chk2)
    finally:
        B.exs_unload_pocket(pid)
