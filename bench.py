#!/usr/bin/env python3
"""Docking throughput on one MI355X: ligand-pocket docks/s.

A step is one pass of the whole hot path over one batch: exs_dock_batch on the
uploaded ligands (all orientations placed, torsion and rigid sweeps, scoring,
per-ligand argmin) and exs_get_best_poses into host memory.  Pocket grids and
ligands are resident in HBM before the timed region (loading and upload are not
timed).  Default workload "scale": 10,000 synthetic ligands (20-60 atoms,
0-12 rotatable bonds) against one 96^3 x 8-channel FP32 pocket grid at 0.375 A,
256 orientations x 32 torsion steps, 2 passes, 27 rigid offsets, one launch per
pocket.

Prints ONE JSON line (rank 0) with the metric, a roofline object for the dock
kernel and the FP64 oracle timed on the host cores as a CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, GB/s
VALU_PEAK_TOPS = 39.32           # 256 CU x 64 lanes x 2.4 GHz: FP32 lane-ops/s (non-packed)


def progress(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_counts(binding, batch, search, channels):
    """Per-ligand algorithmic work of the plain method: texel lookups L, pair tests Q and
    rotated atoms Rot (one orientation each; multiply by K).
      L = n + P * (sum_b (S-1) m_b + (T-1) n),  Q = c0 + P * sum_b (S-1) x_b,
      Rot = P * sum_b (S-1) m_b,
    m_b = atoms turning with bond b, x_b = non-excluded (moving, static) pairs, c0 = all
    non-excluded pairs."""
    S_, P, T = search.torsion_steps, search.passes, search.n_offsets
    L = np.zeros(batch.n_ligands); Q = np.zeros(batch.n_ligands); R = np.zeros(batch.n_ligands)
    for l in range(batch.n_ligands):
        lig = batch.ligand(l)
        t = binding.exs_pack_topology(lig, channels)
        ex = t["excl"]
        n = lig.n
        c0 = (n * n - int(ex.sum())) // 2
        lk = float(n) + P * (T - 1) * n
        q = float(c0)
        rot = 0.0
        for b in range(len(lig.rot)):
            mv = t["moving"][b]
            m = int(mv.sum())
            x = int(((~ex[mv])[:, ~mv]).sum())
            lk += P * (S_ - 1) * m
            q += P * (S_ - 1) * x
            rot += P * (S_ - 1) * m
        L[l], Q[l], R[l] = lk, q, rot
    return L, Q, R


def measured_traffic(n_ligands):
    """HBM bytes of one dock launch from the committed FETCH_SIZE / WRITE_SIZE counter runs,
    or None if the dock kernel's source changed since those counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "dock_kernel_scale_traffic.json")) as f:
            rec = json.load(f)
        with open(os.path.join(ROOT, "paper_2110_11644_amd", "csrc", "dock_kernels.inc"), "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != h:
        return None
    return float(rec["hbm_bytes_per_dock"]) * n_ligands


def cpu_baseline(workload, pocket, batch, search, max_ligands=1024, budget_s=20.0):
    """The FP64 oracle as it stands, OpenMP over ligands on the host cores, on a bounded
    prefix of the same workload (chunks of 32 ligands until the time budget is spent)."""
    import oracle as O
    O.build()
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    g = O.Grid.of(pocket)
    prm = O.Params.of(search)
    done, t0 = 0, time.perf_counter()
    while done < min(max_ligands, batch.n_ligands):
        chunk = batch.subset(range(done, min(done + 32, batch.n_ligands)))
        O.dock_batch([g], prm, chunk, threads=cores)
        done += chunk.n_ligands
        progress("cpu baseline: %d ligands, %.1f s" % (done, time.perf_counter() - t0))
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "docks/s", "cores": cores, "kind": "oracle",
            "sample": "first %d ligands of the %s workload (same pocket and search settings), "
                      "FP64 oracle, OpenMP over ligands, %.1f s" % (done, workload, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scale", choices=["scale", "small"])
    ap.add_argument("--ligands", type=int, default=None, help="override the ligand count")
    ap.add_argument("--ppl", type=int, default=0)
    ap.add_argument("--lpw", type=int, default=0)
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import exs_synth as S
    from paper_2110_11644_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4}), flush=True)
        return
    wl = S.WORKLOADS[args.workload]
    s = wl.search
    n_lig = args.ligands or wl.n_ligands
    progress("generating %s: %d ligands" % (wl.name, n_lig))
    pocket = S.make_pocket(wl, 0)
    batch = S.make_ligand_batch(wl, 0, n_lig)
    stream = torch.cuda.current_stream()
    storage = B.STORAGE[args.storage]
    pid = B.exs_load_pocket_grid(pocket.values, pocket.spacing, pocket.origin, storage, stream=stream)
    bid = B.exs_upload_ligands(batch, pocket_ids=[pid], stream=stream)
    flags = B.EXS_FLAG_PERSISTENT if args.persistent else 0
    prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                          s.clash_cutoff, s.clash_penalty, top_k=0, poses_per_lane=args.ppl,
                          ligands_per_wg=args.lpw, flags=flags)
    L, A = batch.n_ligands, int(batch.atom_offset[-1])

    def step():
        job = B.exs_dock_batch(bid, prm, stream=stream)
        out = B.exs_get_best_poses(job, L, A, coords=True)
        ms = B.exs_job_elapsed_ms(job)
        B.exs_release_job(job)
        return ms, out

    for w in range(args.warmup):
        ms, _ = step()
        progress("warmup %d: dock kernel %.1f ms" % (w, ms))
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ms, out = step()
        kernel_ms.append(ms)
        progress("step %d: dock kernel %.1f ms" % (i, ms))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = L * args.steps / dt
    assert np.all(np.isfinite(out["best_score"]))

    # roofline of the dock kernel: algorithmic texel bytes and FP32 lane-ops per launch
    progress("counting algorithmic work")
    Lk, Qk, Rk = algorithmic_counts(B, batch, s, pocket.channels)
    K = s.n_orient
    tex_bytes = 8.0 * 4.0 * K * Lk.sum() * (0.5 if storage else 1.0)
    ops = K * (30.0 * Lk.sum() + 7.0 * Qk.sum() + 15.0 * Rk.sum())
    kms = float(np.mean(kernel_ms))
    gbs = tex_bytes / (kms * 1e-3) / 1e9
    tops = ops / (kms * 1e-3) / 1e12
    mem = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
    alu = {"bound": "alu", "achieved": round(tops, 2), "peak": VALU_PEAK_TOPS, "unit": "TFLOP/s",
           "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": None}
    traffic = measured_traffic(L) if (args.workload == "scale" and storage == 0 and args.ppl in (0, 1)
                                      and args.lpw in (0, 1) and not args.persistent) else None
    mem["traffic"] = traffic
    alu["traffic"] = traffic
    roof, other = (mem, alu) if mem["frac"] >= alu["frac"] else (alu, mem)
    roof = dict(roof)
    roof["kernel"] = "exs::dock_kernel"
    roof["kernel_ms"] = round(kms, 3)
    roof["other"] = other

    cpu = None
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        cpu = cpu_baseline(wl.name, pocket, batch, s)

    B.exs_release_ligands(bid)
    B.exs_unload_pocket(pid)
    line = {
        "metric": "ligand-pocket docks/sec on 1 MI355X",
        "value": round(value, 2),
        "unit": "docks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if storage == 0 else ("bf16->f32" if storage == 1 else "f16->f32"),
        "data": "synthetic",
        "config": {
            "workload": "%s: %d ligands x 1 pocket %d^3 x %d ch at %.3f A (%s texels); K=%d "
                        "orientations, S=%d torsion steps, P=%d passes, T=%d offsets; %s" % (
                            wl.name, L, pocket.n, pocket.channels, pocket.spacing, args.storage,
                            K, s.torsion_steps, s.passes, s.n_offsets,
                            "one persistent launch" if args.persistent else "one launch per pocket"),
            "ligands": L, "atoms": A, "parallelism": "single GPU",
            "poses_per_lane": args.ppl, "ligands_per_wg": args.lpw,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
