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


def algorithmic_counts(binding, batch, search, channels, with_c0=False):
    """Per-ligand algorithmic work (one orientation each; multiply by K): texel lookups L,
    pair tests Q and turned atom positions Rot.
      L = n + P * (sum_b (S-1) m_b + (T-1) n),  Q = c0 + P * sum_b x_b,
      Rot = P * sum_b (S-1) m_b,
    m_b = atoms turning with bond b, x_b = non-excluded (moving, static) pairs, c0 = all
    non-excluded pairs.  A (moving, static) pair is tested once per bond: its distance over
    all S turns is one closed form (the clashing turns form one arc)."""
    S_, P, T = search.torsion_steps, search.passes, search.n_offsets
    L = np.zeros(batch.n_ligands); Q = np.zeros(batch.n_ligands); R = np.zeros(batch.n_ligands)
    C0 = np.zeros(batch.n_ligands)
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
            q += P * x
            rot += P * (S_ - 1) * m
        L[l], Q[l], R[l], C0[l] = lk, q, rot, c0
    if with_c0:
        return L, Q, R, C0
    return L, Q, R


def kernel_source_sha256():
    """SHA-256 of the dock kernel's sources (the search and its texel gathers)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("dock_kernels.inc", "texel_gather.inc"):
        with open(os.path.join(ROOT, "paper_2110_11644_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(n_ligands):
    """HBM bytes of one dock launch from the committed FETCH_SIZE / WRITE_SIZE counter runs,
    or None if the dock kernel's source changed since those counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "dock_kernel_scale_traffic.json")) as f:
            rec = json.load(f)
        h = kernel_source_sha256()
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
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return {"value": done / dt, "unit": "docks/s", "cores": cores, "kind": "oracle",
            "cpu_model": model,
            "sample": "first %d ligands of the %s workload (same pocket and search settings), "
                      "FP64 oracle, OpenMP over ligands, %.1f s" % (done, workload, dt)}


def roofline_of(B, batch, search, channels, kernel_ms, storage, sample_every=1, traffic=None):
    """Roofline objects of one launch over `batch`: algorithmic texel bytes (8 corners per lookup)
    against the HBM peak, and FP32 lane-ops against the VALU peak; the counts come from every
    `sample_every`-th ligand, scaled.  `traffic`: measured HBM bytes of the launch, if known.

    The texel bytes are served from L2 and the last-level cache more than from HBM (measured
    HBM traffic is about 0.4x of them), so the texel figure is a rate of bytes served by the
    gather path held against the HBM peak; "dram" gives the HBM side from the counters."""
    idx = list(range(0, batch.n_ligands, sample_every))
    sub = batch if sample_every == 1 else batch.subset(idx)
    Lk, Qk, Rk, C0 = algorithmic_counts(B, sub, search, channels, with_c0=True)
    scale = batch.n_ligands / sub.n_ligands
    K, S_ = search.n_orient, search.torsion_steps
    tex_bytes = 8.0 * (4.0 if storage == 0 else 2.0) * K * Lk.sum() * scale
    ops = K * (30.0 * Lk.sum() + 14.0 * Qk.sum() + 6.0 * Rk.sum()) * scale
    # the same work with every (moving, static) pair tested at each of the S-1 turns
    q_turns = C0.sum() + (S_ - 1) * (Qk.sum() - C0.sum())
    ops_turns = K * (30.0 * Lk.sum() + 7.0 * q_turns + 15.0 * Rk.sum()) * scale
    sec = kernel_ms * 1e-3
    gbs = tex_bytes / sec / 1e9
    tops = ops / sec / 1e12
    mem = {"bound": "texel-gather", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
           "ceiling": "MI355X HBM peak (8 TB/s) held against the algorithmic texel bytes, which "
                      "the gathers take from L2 / last-level cache / HBM"}
    if traffic:
        mem["dram"] = {"achieved": round(traffic / sec / 1e9, 3), "unit": "GB/s",
                       "frac": round(traffic / sec / 1e9 / HBM_PEAK_GBS, 4)}
    alu = {"bound": "alu", "achieved": round(tops, 2), "peak": VALU_PEAK_TOPS,
           "unit": "TFLOP/s", "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": traffic,
           "frac_if_every_turn_tested": round(ops_turns / sec / 1e12 / VALU_PEAK_TOPS, 4)}
    roof, other = (mem, alu) if mem["frac"] >= alu["frac"] else (alu, mem)
    roof = dict(roof)
    roof["kernel"] = "exs::dock_kernel"
    roof["kernel_ms"] = round(kernel_ms, 3)
    roof["other"] = other
    if sample_every > 1:
        roof["counts_sampled_every"] = sample_every
    return roof


def gather_probe(B, pid, storage, stream, batch, search, channels, kernel_ms,
                 lanes=256 * 1024, per_lane=256):
    """Lookup rate of the texel-gather probe (the docking lookup alone, independent random
    points) on the same pocket, for two footprints: a 6 A cube around the centre (its texel
    blocks fit an XCD's L2) and a 20 A cube (pocket-wide, beyond L2); the best of 8 or 16
    lookups in flight per lane.  Beside it the dock kernel's own lookup rate."""
    sub = batch.subset(range(0, batch.n_ligands, 10))
    Lk, _, _ = algorithmic_counts(B, sub, search, channels)
    dock_lookups = search.n_orient * Lk.sum() * batch.n_ligands / sub.n_ligands
    out = {"lookups_per_launch": lanes * per_lane,
           "texel_bytes_per_lookup": 32 if storage == 0 else 16}
    # independent points in a 6 A and a 20 A cube; walks in the 6 A cube with steps of at most
    # 0.1 / 0.25 A per axis (the docking lookups' locality: the turns of an atom lie 0.27 A apart
    # on a circle, the 27 offsets of an atom in a 1 A cube)
    for name, half, walk in (("cube_6A", 3.0, 0.0), ("cube_20A", 10.0, 0.0),
                             ("walk_0.25A", 3.0, 0.25), ("walk_0.1A", 3.0, 0.1)):
        best = None
        for nb in (8, 16):
            B.exs_gather_probe(pid, lanes, per_lane, half, walk, 7, batch=nb, stream=stream)   # warm
            ms, _ = B.exs_gather_probe(pid, lanes, per_lane, half, walk, 11, batch=nb, stream=stream)
            rate = lanes * per_lane / (ms * 1e-3)
            if best is None or rate > best[1]:
                best = (ms, rate, nb)
        out[name] = {"ms": round(best[0], 3), "lookups_per_s": round(best[1], 0), "in_flight": best[2]}
    out["dock_lookups_per_s"] = round(dock_lookups / (kernel_ms * 1e-3), 0)
    for name in ("cube_6A", "cube_20A", "walk_0.25A", "walk_0.1A"):
        out["dock_frac_of_" + name] = round(out["dock_lookups_per_s"] / out[name]["lookups_per_s"], 3)
    top = max(("cube_6A", "cube_20A", "walk_0.25A", "walk_0.1A"), key=lambda n: out[n]["lookups_per_s"])
    out["ceiling"] = top
    out["dock_frac_of_ceiling"] = out["dock_frac_of_" + top]
    progress("gather probe: %s" % out)
    return out


def load_batched_pockets(S, B, storage, stream, log=True, pockets=None):
    wl = S.BATCHED
    if pockets is None:
        pockets = S.make_pockets(wl)
    pids = [B.exs_load_pocket_grid(p.values, p.spacing, p.origin, storage, stream=stream)
            for p in pockets]
    if log:
        progress("loaded %d pockets, edges %s" % (len(pids), [p.n for p in pockets]))
    return pockets, pids


def timed_steps(B, torch, bid, prm, L, A, steps, warmup, stream, top_k=0):
    def step():
        job = B.exs_dock_batch(bid, prm, stream=stream)
        out = B.exs_get_best_poses(job, L, A, top_k=top_k, coords=True)
        ms = B.exs_job_elapsed_ms(job)
        B.exs_release_job(job)
        return ms, out
    for w in range(warmup):
        ms, _ = step()
        progress("warmup %d: %.1f ms" % (w, ms))
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    out = None
    for i in range(steps):
        ms, out = step()
        kms.append(ms)
        progress("step %d: %.1f ms" % (i, ms))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, float(np.mean(kms)), out


def run_batched(args, torch, S, B):
    """Uneven ligands over the 15 resident pockets in one persistent launch captured in a
    hipGraph; tile from the autotuner (--tune) or --ppl / --lpw."""
    from paper_2110_11644_amd import autotune
    wl, s = S.BATCHED, S.BATCHED.search
    stream = torch.cuda.current_stream()
    storage = B.STORAGE[args.storage]
    pockets, pids = load_batched_pockets(S, B, storage, stream)
    L = args.ligands or wl.n_ligands
    progress("generating %d ligands" % L)
    batch = S.make_ligand_batch(wl, 0, L)
    bid = B.exs_upload_ligands(batch, pocket_ids=pids, stream=stream)
    flags = B.EXS_FLAG_PERSISTENT | B.EXS_FLAG_GRAPH
    ppl, lpw, tuned = args.ppl or 1, args.lpw or 1, None
    if args.tune:
        # a sample that keeps the full run's work-queue layout: pockets holding more ligands
        # than the device has in flight (3,072 waves) are scheduled pocket by pocket
        inflight = 3072 // -(-s.n_orient // 64)
        n_sample = min(L, max(4096, 2 * inflight * len(pids)))
        sample = batch.subset(range(0, L, max(1, L // n_sample)))
        sid = B.exs_upload_ligands(sample, pocket_ids=pids, stream=stream)
        tuned = autotune.tune(sid, s, storage, B.EXS_FLAG_PERSISTENT,
                              float(np.diff(sample.atom_offset).mean()), use_cache=False,
                              stream=stream, log=progress)
        B.exs_release_ligands(sid)
        ppl, lpw = tuned["ppl"], tuned["lpw"]
    prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                          s.clash_cutoff, s.clash_penalty, poses_per_lane=ppl, ligands_per_wg=lpw,
                          flags=flags)
    A = int(batch.atom_offset[-1])
    dt, kms, out = timed_steps(B, torch, bid, prm, L, A, args.steps, args.warmup, stream)
    assert np.all(np.isfinite(out["best_score"]))
    value = L * args.steps / dt
    progress("counting algorithmic work (sampled)")
    roof = roofline_of(B, batch, s, 8, kms, storage, sample_every=max(1, L // 10000))
    B.exs_release_ligands(bid)
    for pid in pids:
        B.exs_unload_pocket(pid)
    line = {
        "metric": "ligand-pocket docks/sec on 1 MI355X (batched)", "value": round(value, 2),
        "unit": "docks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if storage == 0 else args.storage,
        "data": "synthetic",
        "config": {"workload": "batched: %d ligands (log-normal atoms, median 35, 10-90; 0-15 "
                               "rotatable bonds) over 15 resident pockets (edges %s, 8 ch, 0.375 A); "
                               "K=256, S=32, P=2, T=27; one persistent launch in a hipGraph" % (
                                   L, sorted(set(p.n for p in pockets))),
                   "ligands": L, "atoms": A, "poses_per_lane": ppl, "ligands_per_wg": lpw,
                   "tile_timings_ms": None if tuned is None else tuned["timings"],
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def top_set(scores, frac):
    n = max(1, int(round(len(scores) * frac)))
    order = np.lexsort((np.arange(len(scores)), scores))   # score ascending, ties by ligand id
    return set(order[:n].tolist())


def run_precision(args, torch, S, B):
    """BF16 and FP16 texels (FP32 interpolation) with FP64 rescoring of the top 8 poses,
    against the FP32 path (all ligands) and the FP64 oracle (a prefix sample)."""
    import oracle as O
    wl, s = S.BATCHED, S.PRECISION.search
    stream = torch.cuda.current_stream()
    L = args.ligands or wl.n_ligands
    progress("generating %d ligands" % L)
    batch = S.make_ligand_batch(wl, 0, L)
    A = int(batch.atom_offset[-1])
    flags = B.EXS_FLAG_PERSISTENT | B.EXS_FLAG_GRAPH
    results = {}
    pockets = S.make_pockets(wl)
    for name, storage, top_k in (("f32", 0, 0), ("bf16", 1, 8), ("f16", 2, 8)):
        pockets, pids = load_batched_pockets(S, B, storage, stream, log=(name == "f32"),
                                             pockets=pockets)
        bid = B.exs_upload_ligands(batch, pocket_ids=pids, stream=stream)
        prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                              s.clash_cutoff, s.clash_penalty, top_k=top_k,
                              poses_per_lane=args.ppl or 1, ligands_per_wg=args.lpw or 1,
                              flags=flags)
        dt, kms, out = timed_steps(B, torch, bid, prm, L, A, args.steps, args.warmup, stream,
                                   top_k=top_k)
        results[name] = dict(value=L * args.steps / dt, kernel_ms=kms, out=out)
        progress("%s: %.0f docks/s" % (name, results[name]["value"]))
        B.exs_release_ligands(bid)
        for pid in pids:
            B.exs_unload_pocket(pid)
    # FP64 oracle on a prefix sample (best score of each ligand)
    M = min(args.oracle_sample, L)
    progress("oracle on %d ligands" % M)
    grids = [O.Grid.of(p) for p in pockets]
    cores = len(os.sched_getaffinity(0))
    ref = O.dock_batch(grids, O.Params.of(s), batch.subset(range(M)), threads=cores)
    prm_o = O.Params.of(s)
    report = {}
    ref32 = results["f32"]["out"]["best_score"].astype(np.float64)
    for name in ("bf16", "f16"):
        out = results[name]["out"]
        b64 = out["desc"]["score_fp64"].astype(np.float64)
        err = np.abs(b64[:M] - ref["best_score"])
        rel = err / np.maximum(np.abs(ref["best_score"]), 1.0)
        rmsd = []
        same = 0
        for l in range(M):
            lig = batch.ligand(l)
            d = out["desc"][l]
            X = O.pose_from_desc(grids[lig.pocket], prm_o, lig, int(d["orient"]),
                                 d["theta"][:len(lig.rot)], d["tau"])
            a0, a1 = int(batch.atom_offset[l]), int(batch.atom_offset[l + 1])
            rmsd.append(float(np.sqrt(np.mean(np.sum((out["coords"][a0:a1] - X) ** 2, axis=1)))))
            same += int(d["orient"]) == int(ref["best_k"][l])
        report[name] = {
            "docks_per_s": round(results[name]["value"], 1),
            "kernel_ms": round(results[name]["kernel_ms"], 2),
            "score_err_vs_oracle_max": float(err.max()), "score_err_vs_oracle_mean": float(err.mean()),
            "score_relerr_vs_oracle_max": float(rel.max()),
            "best_pose_rmsd_vs_fp64_rebuild_max_A": max(rmsd),
            "best_orientation_equal_to_oracle": same / M,
            "top1pct_overlap_vs_fp32_gpu_all": len(top_set(b64, 0.01) & top_set(ref32, 0.01))
                                               / len(top_set(ref32, 0.01)),
            "top1pct_overlap_vs_oracle_sample": len(top_set(b64[:M], 0.01)
                                                    & top_set(ref["best_score"], 0.01))
                                                / len(top_set(ref["best_score"], 0.01)),
            "top10pct_overlap_vs_oracle_sample": len(top_set(b64[:M], 0.1)
                                                     & top_set(ref["best_score"], 0.1))
                                                 / len(top_set(ref["best_score"], 0.1)),
        }
    f32err = np.abs(ref32[:M] - ref["best_score"]) / np.maximum(np.abs(ref["best_score"]), 1.0)
    line = {
        "metric": "ligand-pocket docks/sec on 1 MI355X (16-bit texels + FP64 top-8 rescoring)",
        "value": round(results["f16"]["value"], 2), "unit": "docks/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16->f32 (+f64 rescoring)", "data": "synthetic",
        "config": {"workload": "precision: the batched inputs (%d ligands, 15 pockets), texels "
                               "BF16 and FP16, top_k=8 FP64 rescoring; FP32 run for reference" % L,
                   "ligands": L, "oracle_sample": M, "parallelism": "single GPU"},
        "fp32_docks_per_s": round(results["f32"]["value"], 1),
        "fp32_relerr_vs_oracle_max": float(f32err.max()),
        "precision": report,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_serving(args, torch, S, B):
    """Poisson arrivals of requests (1-512 ligands, log-uniform, random pocket) at a fixed
    offered load, served by the continuous-batching server; the same trace replayed with one
    plain launch per request (FIFO) for comparison."""
    import threading
    s = S.SERVING.search
    stream = torch.cuda.current_stream()
    storage = B.STORAGE[args.storage]
    pockets, pids = load_batched_pockets(S, B, storage, stream)
    prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                          s.clash_cutoff, s.clash_penalty, poses_per_lane=args.ppl or 1,
                          ligands_per_wg=args.lpw or 1, flags=B.EXS_FLAG_PERSISTENT)
    # capacity: persistent launch over a sample of the request ligands
    cap_batch = S.make_ligand_batch(S.BATCHED, 0, 4096)
    cid = B.exs_upload_ligands(cap_batch, pocket_ids=pids, stream=stream)
    _, cap_ms, _ = timed_steps(B, torch, cid, prm, cap_batch.n_ligands,
                               int(cap_batch.atom_offset[-1]), 2, 1, stream)
    B.exs_release_ligands(cid)
    capacity = cap_batch.n_ligands / (cap_ms * 1e-3)
    warm = max(10, args.requests // 20)   # 100 for the default 2,000 timed requests
    n_req = args.requests + warm
    sweep = [float(x) for x in args.sweep.split(",") if x.strip()] if args.sweep else []
    mean_size = 82.0
    rate = args.load * capacity / mean_size
    trace = S.make_trace(n_req, rate)
    progress("capacity %.0f docks/s, %d requests at %.1f req/s (load %.2f)" % (
        capacity, n_req, rate, args.load))
    reqs = []
    for r in trace:
        ligs = S.serving_ligands(r)
        b = S.batch_from_ligands(ligs)
        b.pocket_id[:] = r.pocket
        reqs.append(b)
    progress("generated %d ligands" % sum(b.n_ligands for b in reqs))

    def replay(submit, finish, time_scale=1.0):
        """Submit at the trace's arrival times (scaled by time_scale); returns per-request
        latency (s) and span."""
        lat = [None] * n_req
        done_t = [None] * n_req
        handles = [None] * n_req
        ready = [threading.Event() for _ in range(n_req)]
        t0 = time.perf_counter()

        def waiter():
            for i in range(n_req):
                ready[i].wait()
                finish(handles[i], reqs[i])
                done_t[i] = time.perf_counter()
                lat[i] = done_t[i] - (t0 + trace[i].arrival_s * time_scale)
        th = threading.Thread(target=waiter)
        th.start()
        for i, r in enumerate(trace):
            now = time.perf_counter() - t0
            if r.arrival_s * time_scale > now:
                time.sleep(r.arrival_s * time_scale - now)
            handles[i] = submit(reqs[i])
            ready[i].set()
        th.join()
        return np.array(lat), t0, done_t

    timed_lig = sum(reqs[i].n_ligands for i in range(warm, n_req))

    def serve(load):
        """The trace at `load` (arrival times scaled) through a fresh server."""
        scale = args.load / load
        srv = B.exs_server_create(pids, prm, hbm_budget_bytes=8 << 30,
                                  max_iter_ligands=args.serve_max_iter,
                                  max_inflight_iters=args.serve_inflight)
        lat, t0, done = replay(
            lambda b: B.exs_server_submit(srv, b, pocket_ids=pids),
            lambda h, b: B.exs_server_poll(srv, h, b.n_ligands, int(b.atom_offset[-1])),
            time_scale=scale)
        st = B.exs_server_get_stats(srv)
        B.exs_server_destroy(srv)
        span = done[-1] - (t0 + trace[warm].arrival_s * scale)
        return lat, span, st

    lat_s, span_s, stats = serve(args.load)
    swept = {}
    for ld in sweep:
        lat_x, span_x, st_x = serve(ld)
        swept["%.2f" % ld] = {"p50_ms": round(float(np.percentile(lat_x[warm:], 50)) * 1e3, 2),
                              "p99_ms": round(float(np.percentile(lat_x[warm:], 99)) * 1e3, 2),
                              "docks_per_s": round(timed_lig / span_x, 1),
                              "iterations": st_x["iterations"]}
        progress("served at load %.2f: %s" % (ld, swept["%.2f" % ld]))
    progress("served: p50 %.1f ms p99 %.1f ms" % (np.percentile(lat_s[warm:], 50) * 1e3,
                                                 np.percentile(lat_s[warm:], 99) * 1e3))
    # plain per-request launch: one upload + dock + fetch per request, in arrival order
    import queue
    q = queue.Queue()
    results = {}

    def plain_worker():
        while True:
            item = q.get()
            if item is None:
                return
            i, b = item
            bid = B.exs_upload_ligands(b, pocket_ids=pids, stream=stream)
            prm_p = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets,
                                    s.offset_step, s.clash_cutoff, s.clash_penalty,
                                    poses_per_lane=args.ppl or 1, ligands_per_wg=args.lpw or 1)
            job = B.exs_dock_batch(bid, prm_p, stream=stream)
            B.exs_get_best_poses(job, b.n_ligands, int(b.atom_offset[-1]))
            B.exs_release_job(job)
            B.exs_release_ligands(bid)
            results[i].set()
    wk = threading.Thread(target=plain_worker)
    wk.start()
    counter = [0]

    def plain_submit(b):
        i = counter[0]
        counter[0] += 1
        results[i] = threading.Event()
        q.put((i, b))
        return i
    lat_p, t0p, done_p = replay(plain_submit, lambda h, b: results[h].wait())
    q.put(None)
    wk.join()
    for pid in pids:
        B.exs_unload_pocket(pid)
    span_p = done_p[-1] - (t0p + trace[warm].arrival_s)
    line = {
        "metric": "ligand-pocket docks/sec on 1 MI355X (served), p50/p99 latency",
        "value": round(timed_lig / span_s, 2), "unit": "docks/s", "n_gpus": 1,
        "steps": args.requests, "warmup": warm, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if storage == 0 else args.storage, "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals at %.2f x capacity (%.0f docks/s), "
                               "requests of 1-512 ligands (log-uniform) against one of 15 resident "
                               "pockets; continuous batching vs one plain launch per request" % (
                                   args.load, capacity),
                   "requests": args.requests, "warmup_requests": warm,
                   "ligands": timed_lig, "parallelism": "single GPU"},
        "served": {"p50_ms": round(float(np.percentile(lat_s[warm:], 50)) * 1e3, 2),
                   "p99_ms": round(float(np.percentile(lat_s[warm:], 99)) * 1e3, 2),
                   "docks_per_s": round(timed_lig / span_s, 1), "iterations": stats["iterations"]},
        "served_other_loads": swept,
        "plain_per_request": {"p50_ms": round(float(np.percentile(lat_p[warm:], 50)) * 1e3, 2),
                              "p99_ms": round(float(np.percentile(lat_p[warm:], 99)) * 1e3, 2),
                              "docks_per_s": round(timed_lig / span_p, 1)},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_campaign(args, torch, S, B):
    """A screening campaign on one GPU (the paper's pipeline of Sec. 3.2 on one device) through
    exs_campaign_run: the batched library validated and costed on host threads, cut most costly
    first into chunks that packer threads submit to the serving engine while earlier chunks
    dock, every ligand's best score scattered back, the top-1 % hits kept.  The value is
    end-to-end docks/s from raw host ligands to hits in host memory."""
    wl, s = S.BATCHED, S.BATCHED.search
    stream = torch.cuda.current_stream()
    storage = B.STORAGE[args.storage]
    pockets, pids = load_batched_pockets(S, B, storage, stream)
    L = args.ligands or wl.n_ligands
    progress("generating %d ligands (the library stand-in; not timed)" % L)
    library = S.make_ligand_batch(wl, 0, L)
    prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                          s.clash_cutoff, s.clash_penalty, poses_per_lane=1, ligands_per_wg=1,
                          flags=B.EXS_FLAG_PERSISTENT)
    t0 = time.perf_counter()
    res = B.exs_campaign_run(pids, prm, library, chunk_ligands=args.chunk, packers=args.packers,
                             hit_fraction=0.01, hbm_budget_bytes=16 << 30,
                             max_iter_ligands=args.max_iter, library_pocket_ids=pids)
    dt = time.perf_counter() - t0
    for pid in pids:
        B.exs_unload_pocket(pid)
    best, hits = res["best_score"], res["hits"]
    assert np.all(np.isfinite(best))
    golden = golden_oracle()
    line = {
        "metric": "ligand-pocket docks/sec on 1 MI355X (campaign, end to end)",
        "value": round(L / dt, 2), "unit": "docks/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if storage == 0 else args.storage, "data": "synthetic",
        "config": {"workload": "campaign: the batched library (%d ligands, 15 pockets) cut most "
                               "costly first into chunks of %d, streamed through the serving "
                               "engine by %d packer threads; top-1 %% hits kept" % (
                                   L, args.chunk, args.packers),
                   "ligands": L, "chunk": args.chunk, "packers": args.packers,
                   "max_iter": args.max_iter, "parallelism": "single GPU"},
        "campaign": res["stats"], "hits": len(hits), "best_hit_score": float(best[hits[0]]),
        "vs_oracle": None if golden is None or L < len(golden["best_score"])
        else vs_oracle(best, golden),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_batched_20k.npz")


def golden_oracle():
    """FP64 oracle best scores of the first 20,000 batched ligands (written by
    tests/golden/make_oracle_batched.py, which calls only the oracle), or None."""
    try:
        z = np.load(GOLDEN)
    except OSError:
        return None
    return {"best_score": z["best_score"], "near_tie_best": z["near_tie_best"]}


def vs_oracle(best, golden):
    """Top-1 % hit overlap and score error of GPU best scores (ligands 0..) against the oracle's
    best scores of the declared subset."""
    ref = golden["best_score"]
    m = len(ref)
    got = np.asarray(best[:m], np.float64)
    hits = top_set(ref, 0.01)
    err = np.abs(got - ref)
    rel = err / np.maximum(np.abs(ref), 1.0)
    return {"subset": m, "hits": len(hits),
            "top1pct_overlap": round(len(top_set(got, 0.01) & hits) / len(hits), 4),
            "score_abs_err_max": round(float(err.max()), 6),
            "score_abs_err_mean": round(float(err.mean()), 6),
            "score_rel_err_max": round(float(rel.max()), 8),
            "within_1e-4_rel": round(float(np.mean(rel <= 1e-4)), 4)}


def replay(trace, reqs, submit, finish, time_scale=1.0):
    """Submit each request at its trace arrival time (scaled); a waiter thread finishes them in
    order.  Returns per-request latency (s), the start time and the completion times."""
    import threading
    n = len(trace)
    lat, done_t, handles = [None] * n, [None] * n, [None] * n
    ready = [threading.Event() for _ in range(n)]
    t0 = time.perf_counter()

    def waiter():
        for i in range(n):
            ready[i].wait()
            finish(handles[i], reqs[i])
            done_t[i] = time.perf_counter()
            lat[i] = done_t[i] - (t0 + trace[i].arrival_s * time_scale)
    th = threading.Thread(target=waiter)
    th.start()
    for i, r in enumerate(trace):
        now = time.perf_counter() - t0
        if r.arrival_s * time_scale > now:
            time.sleep(r.arrival_s * time_scale - now)
        handles[i] = submit(reqs[i])
        ready[i].set()
    th.join()
    return np.array(lat), t0, done_t


def serve_trace(B, pids, prm, trace, reqs, warm, time_scale=1.0, budget=8 << 30):
    """The trace through a fresh continuous-batching server: latency percentiles and served
    docks/s over the requests after the first `warm`."""
    srv = B.exs_server_create(pids, prm, hbm_budget_bytes=budget)
    try:
        lat, t0, done = replay(
            trace, reqs, lambda b: B.exs_server_submit(srv, b, pocket_ids=pids),
            lambda h, b: B.exs_server_poll(srv, h, b.n_ligands, int(b.atom_offset[-1])),
            time_scale)
        st = B.exs_server_get_stats(srv)
    finally:
        B.exs_server_destroy(srv)
    timed = sum(reqs[i].n_ligands for i in range(warm, len(reqs)))
    span = done[-1] - (t0 + trace[warm].arrival_s * time_scale)
    return {"p50_ms": round(float(np.percentile(lat[warm:], 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat[warm:], 99)) * 1e3, 2),
            "docks_per_s": round(timed / span, 1), "iterations": st["iterations"]}


def plain_trace(B, torch, pids, prm, trace, reqs, warm, workers):
    """The trace with one plain launch per request (upload + dock + fetch), FIFO, served by
    `workers` host threads each on its own HIP stream (several GPU workers per device)."""
    import queue
    import threading
    q = queue.Queue()
    events = {}

    def worker():
        st = torch.cuda.Stream()
        while True:
            item = q.get()
            if item is None:
                return
            i, b = item
            bid = B.exs_upload_ligands(b, pocket_ids=pids, stream=st)
            job = B.exs_dock_batch(bid, prm, stream=st)
            B.exs_get_best_poses(job, b.n_ligands, int(b.atom_offset[-1]))
            B.exs_release_job(job)
            B.exs_release_ligands(bid)
            events[i].set()
    ths = [threading.Thread(target=worker) for _ in range(workers)]
    for t in ths:
        t.start()
    counter = [0]

    def submit(b):
        i = counter[0]
        counter[0] += 1
        events[i] = threading.Event()
        q.put((i, b))
        return i
    try:
        lat, t0, done = replay(trace, reqs, submit, lambda h, b: events[h].wait())
    finally:
        for _ in ths:
            q.put(None)
        for t in ths:
            t.join()
    timed = sum(reqs[i].n_ligands for i in range(warm, len(reqs)))
    span = done[-1] - (t0 + trace[warm].arrival_s)
    return {"workers": workers, "p50_ms": round(float(np.percentile(lat[warm:], 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat[warm:], 99)) * 1e3, 2),
            "docks_per_s": round(timed / span, 1)}


def trace_requests(S, n_req, rate):
    """Poisson trace of n_req requests and their ligand batches (one pass of the generator)."""
    trace = S.make_trace(n_req, rate)
    total = sum(r.size for r in trace)
    ligs = S.make_ligands(S.SERVING, 0, total)
    reqs = []
    for r in trace:
        part = ligs[r.ligand_start:r.ligand_start + r.size]
        for l in part:
            l.pocket = r.pocket
        reqs.append(S.batch_from_ligands(part))
    return trace, reqs


def batched_launch(B, torch, pids, batch, s, storage, top_k, steps, warmup, stream, flags):
    """Timed launches of the whole batch: docks/s, mean kernel time (HIP events on the job's
    stream) and the best-pose output of the last step."""
    prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                          s.clash_cutoff, s.clash_penalty, top_k=top_k, poses_per_lane=1,
                          ligands_per_wg=1, flags=flags)
    bid = B.exs_upload_ligands(batch, pocket_ids=pids, stream=stream)
    try:
        dt, kms, out = timed_steps(B, torch, bid, prm, batch.n_ligands,
                                   int(batch.atom_offset[-1]), steps, warmup, stream, top_k=top_k)
    finally:
        B.exs_release_ligands(bid)
    return batch.n_ligands * steps / dt, kms, dt / steps, out


def method_work(binding, batch, search, channels, clusters, keep, unfold_passes):
    """Algorithmic lane-ops of the method's other steps, summed over the ligands (FP32 for the
    unfolding and the ranking, FP64 for the second-stage rescoring; both run at one lane-op per
    lane and cycle on the vector ALU):
      unfolding  passes * sum_b S * m_b * (9 (n - m_b) + 12)
                 (S turn positions of each moving atom, 12 lane-ops each, and its distance to
                 every static atom, 9: three differences, three products, root, sum);
      ranking    K^2 (rank of each pose by score) + 2 * K * c * 3n
                 (each pose against each of the c leaders: a difference and an fma per row);
      rescoring  keep * (30 n + 12 c0 + 40 B + 20 (n + sum_b m_b))
                 (per pose: n FP64 trilinear lookups, c0 contact pairs, B torsion terms and the
                 FP64 rebuild).
    m_b = atoms turning with bond b, c0 = non-excluded pairs, c = the ligand's clusters."""
    S_, K = search.torsion_steps, search.n_orient
    unf = rank = res = 0.0
    for l in range(batch.n_ligands):
        lig = batch.ligand(l)
        t = binding.exs_pack_topology(lig, channels)
        n = lig.n
        c0 = (n * n - int(t["excl"].sum())) // 2
        ms = [int(t["moving"][b].sum()) for b in range(len(lig.rot))]
        unf += unfold_passes * sum(S_ * m * (9 * (n - m) + 12) for m in ms)
        rank += K * K + 2.0 * K * float(clusters[l]) * 3 * n
        res += keep * (30 * n + 12 * c0 + 40 * len(ms) + 20 * (n + sum(ms)))
    return {"unfold": unf, "rank": rank, "rescore2": res}


def step_roofline(ops, ms):
    tops = ops / (ms * 1e-3) / 1e12
    return {"ms": round(ms, 3), "bound": "alu", "lane_ops": float(ops), "achieved": round(tops, 3),
            "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s", "frac": round(tops / VALU_PEAK_TOPS, 4)}


def method_steps_leg(B, torch, S, pid, s, stream, n=3000):
    """The method's other steps on the first `n` scale ligands (Sec. 3.1): unfolding of the
    input conformations (S = 32, 2 passes; host wall time of the call), then one dock job as
    it is and one that also ranks each ligand's final poses (3 A clusters, 30 kept) and rescores
    the ranked poses with the second-stage score (HIP-event times of the job, median of 3)."""
    batch = S.make_ligand_batch(S.WORKLOADS["scale"], 0, n)
    L, A = batch.n_ligands, int(batch.atom_offset[-1])
    bid = B.exs_upload_ligands(batch, pocket_ids=[pid], stream=stream)
    try:
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        B.exs_unfold_ligands(bid, s.torsion_steps, 2, stream=stream)
        e1.record(stream)
        unfold_ms = (time.perf_counter() - t0) * 1e3
        e1.synchronize()
        unfold_kernel_ms = e0.elapsed_time(e1)   # the kernel, bracketed on its own stream

        def job_ms(prm, ranked):
            ms, nc, stages = [], None, []
            for _ in range(4):
                job = B.exs_dock_batch(bid, prm, stream=stream)
                B.exs_get_best_poses(job, L, A)
                if ranked:
                    nc, _ = B.exs_get_ranked_poses(job, L, 30)
                    B.exs_get_rescored_poses(job, L, 30)
                    stages.append(B.exs_job_stage_ms(job))
                ms.append(B.exs_job_elapsed_ms(job))
                B.exs_release_job(job)
            med = {k: float(np.median([st[k] for st in stages[1:]])) for k in ("rank", "rescore2")} \
                if ranked else None
            return float(np.median(ms[1:])), nc, med

        plain = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                                s.clash_cutoff, s.clash_penalty)
        ranked = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                                 s.clash_cutoff, s.clash_penalty, flags=B.EXS_FLAG_RESCORE2,
                                 cluster_rmsd_A=3.0, rank_keep=30)
        dock_ms, _, _ = job_ms(plain, False)
        full_ms, nc, st_ms = job_ms(ranked, True)
    finally:
        B.exs_release_ligands(bid)
    work = method_work(B, batch, s, S.WORKLOADS["scale"].channels, nc, 30, 2)
    return {"ligands": L, "unfold_ms": round(unfold_ms, 3), "dock_ms": round(dock_ms, 3),
            "dock_rank_rescore2_ms": round(full_ms, 3),
            "rank_rescore2_ms": round(full_ms - dock_ms, 3),
            "clusters_mean": round(float(nc.mean()), 2),
            "roofline": {"unfold": step_roofline(work["unfold"], unfold_kernel_ms),
                         "rank": step_roofline(work["rank"], st_ms["rank"]),
                         "rescore2": step_roofline(work["rescore2"], st_ms["rescore2"])},
            "steps": "unfold (S=32, 2 passes), dock, rank (3 A, keep 30), second-stage rescoring"}


def driver_legs(args, torch, S, B):
    """The rest of the headline metric, under the same run: the batched workload (100,000
    ligands over 15 resident pockets) as one persistent launch in a hipGraph, FP32 and with
    16-bit texels + FP64 top-8 rescoring, beside the plain FP32 one-launch-per-pocket form, with
    top-1 % hit overlap against the FP64 oracle's best scores of the first 20,000 ligands; and
    the serving workload (Poisson arrivals at 0.7 x capacity), FP32 and BF16 + top-8, against
    one plain launch per request from several workers."""
    wl, s = S.BATCHED, S.BATCHED.search
    stream = torch.cuda.current_stream()
    steps = max(1, min(args.steps, args.extra_steps))
    warm = max(1, min(args.warmup, 2))
    progress("batched: generating 15 pockets and %d ligands" % wl.n_ligands)
    pockets = S.make_pockets(wl)
    batch = S.make_ligand_batch(wl, 0, args.ligands_batched or wl.n_ligands)
    L = batch.n_ligands
    golden = golden_oracle()
    persist = B.EXS_FLAG_PERSISTENT | B.EXS_FLAG_GRAPH
    out = {"workload": "batched: %d ligands (log-normal atoms, median 35, 10-90; 0-15 rotatable "
                       "bonds) over 15 resident pockets (edges %s, 8 ch, 0.375 A); K=256, S=32, "
                       "P=2, T=27" % (L, sorted(set(p.n for p in pockets))),
           "steps": steps, "warmup": warm,
           "oracle_subset": None if golden is None else
           "FP64 oracle best scores of ligands 0..19,999 (tests/golden/oracle_batched_20k.npz)"}
    legs = {}
    for name, storage, top_k, flags in (("plain_f32_per_pocket", 0, 0, 0),
                                        ("persistent_f32", 0, 0, persist),
                                        ("persistent_f32_top8", 0, 8, persist),
                                        ("persistent_bf16_top8", 1, 8, persist),
                                        ("persistent_f16_top8", 2, 8, persist)):
        pids = [B.exs_load_pocket_grid(p.values, p.spacing, p.origin, storage, stream=stream)
                for p in pockets]
        try:
            v, kms, step_s, res = batched_launch(B, torch, pids, batch, s, storage, top_k, steps,
                                                 warm, stream, flags)
        finally:
            for pid in pids:
                B.exs_unload_pocket(pid)
        best = res["desc"]["score_fp64"] if top_k else res["best_score"]
        leg = {"docks_per_s": round(v, 1), "ms_per_step": round(step_s * 1e3, 3),
               "kernel_ms": round(kms, 3), "texels": ("f32", "bf16", "f16")[storage],
               "top_k_fp64": top_k,
               "launch": "one launch per pocket" if not flags else "persistent + hipGraph"}
        if flags:
            leg["roofline"] = roofline_of(B, batch, s, 8, kms, storage, sample_every=max(1, L // 10000))
        if golden is not None and L >= len(golden["best_score"]):
            leg["vs_oracle"] = vs_oracle(best, golden)
        legs[name] = leg
        progress("batched %s: %s" % (name, {k: leg[k] for k in ("docks_per_s", "kernel_ms")}))
    out["legs"] = legs
    # campaign: the same library from host memory to the hit list through exs_campaign_run
    pids = [B.exs_load_pocket_grid(p.values, p.spacing, p.origin, 0, stream=stream) for p in pockets]
    try:
        prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                              s.clash_cutoff, s.clash_penalty, poses_per_lane=1, ligands_per_wg=1,
                              flags=B.EXS_FLAG_PERSISTENT)
        t0 = time.perf_counter()
        res = B.exs_campaign_run(pids, prm, batch, chunk_ligands=16384, packers=args.packers,
                                 hit_fraction=0.01, hbm_budget_bytes=16 << 30,
                                 max_iter_ligands=16384, library_pocket_ids=pids)
        dt = time.perf_counter() - t0
    finally:
        for pid in pids:
            B.exs_unload_pocket(pid)
    camp = {"docks_per_s": round(L / dt, 1), "seconds": round(dt, 4),
            "texels": "f32", "chunk": 16384, "packers": args.packers,
            "workload": "the batched library from host memory: validated and costed on host "
                        "threads, cut pocket by pocket into chunks streamed through the serving "
                        "engine, top-1 % hits kept"}
    if golden is not None and L >= len(golden["best_score"]):
        camp["vs_oracle"] = vs_oracle(res["best_score"], golden)
    out["campaign"] = camp
    progress("campaign: %s" % {k: camp[k] for k in ("docks_per_s", "seconds")})
    # serving: Poisson arrivals at args.load x the persistent FP32 capacity
    cap = legs["persistent_f32"]["docks_per_s"]
    n_req = args.requests + args.requests // 20
    rate = args.load * cap / 82.0
    progress("serving: generating %d requests" % n_req)
    trace, reqs = trace_requests(S, n_req, rate)
    warm_req = args.requests // 20
    srv = {"load": args.load, "capacity_docks_per_s": cap, "requests": args.requests,
           "warmup_requests": warm_req,
           "ligands": sum(r.n_ligands for r in reqs[warm_req:]),
           "trace": "Poisson arrivals, 1-512 ligands per request (log-uniform), one of 15 "
                    "resident pockets each"}
    for name, storage, top_k in (("served_f32", 0, 0), ("served_bf16_top8", 1, 8)):
        pids = [B.exs_load_pocket_grid(p.values, p.spacing, p.origin, storage, stream=stream)
                for p in pockets]
        try:
            prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets,
                                  s.offset_step, s.clash_cutoff, s.clash_penalty, top_k=top_k,
                                  poses_per_lane=1, ligands_per_wg=1, flags=B.EXS_FLAG_PERSISTENT)
            srv[name] = serve_trace(B, pids, prm, trace, reqs, warm_req)
            progress("%s: %s" % (name, srv[name]))
            if storage == 1:
                # the same requests at 0.7 x the mixed-precision form's own capacity (arrival
                # times compressed by the ratio of the capacities)
                own = legs["persistent_bf16_top8"]["docks_per_s"]
                srv[name + "_own_load"] = dict(
                    serve_trace(B, pids, prm, trace, reqs, warm_req, time_scale=cap / own),
                    offered_docks_per_s=round(args.load * own, 1))
                progress("%s at its own load: %s" % (name, srv[name + "_own_load"]))
            if storage == 0:
                prm_p = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets,
                                        s.offset_step, s.clash_cutoff, s.clash_penalty,
                                        poses_per_lane=1, ligands_per_wg=1)
                srv["plain_per_request_f32"] = plain_trace(B, torch, pids, prm_p, trace, reqs,
                                                           warm_req, args.plain_workers)
                progress("plain per request: %s" % srv["plain_per_request_f32"])
        finally:
            for pid in pids:
                B.exs_unload_pocket(pid)
    out["serving"] = srv
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scale",
                    choices=["scale", "small", "batched", "precision", "serving", "campaign"])
    ap.add_argument("--tune", action="store_true", help="autotune the tile (batched)")
    ap.add_argument("--chunk", type=int, default=16384, help="campaign: ligands per request")
    ap.add_argument("--packers", type=int, default=4, help="campaign: host packing threads")
    ap.add_argument("--max-iter", type=int, default=16384,
                    help="campaign: ligands per server iteration (0 = the server's default)")
    ap.add_argument("--rank-keep", type=int, default=0,
                    help="scale/small: rank each ligand's final poses and keep this many (0 = off)")
    ap.add_argument("--cluster-rmsd", type=float, default=3.0, help="ranking: RMSD threshold (A)")
    ap.add_argument("--rescore2", action="store_true",
                    help="scale/small with --rank-keep: rescore the ranked poses (second stage)")
    ap.add_argument("--unfold-passes", type=int, default=0,
                    help="scale/small: unfold the ligands first (passes; 0 = off), timed apart")
    ap.add_argument("--requests", type=int, default=1000, help="serving: timed requests")
    ap.add_argument("--sweep", default="0.5,0.9", help="serving: other offered loads to serve")
    ap.add_argument("--serve-max-iter", type=int, default=0,
                    help="serving workload: ligands per server iteration (0 = the server's default)")
    ap.add_argument("--serve-inflight", type=int, default=0,
                    help="serving workload: iterations in flight, 1 or 2 (0 = the server's default)")
    ap.add_argument("--load", type=float, default=0.7, help="serving: offered load / capacity")
    ap.add_argument("--oracle-sample", type=int, default=192,
                    help="precision: ligands checked against the FP64 oracle")
    ap.add_argument("--ligands", type=int, default=None, help="override the ligand count")
    ap.add_argument("--ppl", type=int, default=0)
    ap.add_argument("--lpw", type=int, default=0)
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="scale: skip the batched / precision / serving legs of the default run")
    ap.add_argument("--extra-steps", type=int, default=3,
                    help="timed steps of each batched leg (at most --steps)")
    ap.add_argument("--ligands-batched", type=int, default=None,
                    help="ligands of the batched legs (default: the workload's 100,000)")
    ap.add_argument("--plain-workers", type=int, default=4,
                    help="host workers (one HIP stream each) of the plain per-request baseline")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
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
    if args.workload == "batched":
        return run_batched(args, torch, S, B)
    if args.workload == "precision":
        return run_precision(args, torch, S, B)
    if args.workload == "serving":
        return run_serving(args, torch, S, B)
    if args.workload == "campaign":
        return run_campaign(args, torch, S, B)
    wl = S.WORKLOADS[args.workload]
    s = wl.search
    n_lig = args.ligands or wl.n_ligands
    progress("generating %s: %d ligands" % (wl.name, n_lig))
    pocket = S.make_pocket(wl, 0)
    batch = S.make_ligand_batch(wl, 0, n_lig)
    stream = torch.cuda.current_stream()
    storage = B.STORAGE[args.storage]
    pid = B.exs_load_pocket_grid(pocket.values, pocket.spacing, pocket.origin, storage, stream=stream)
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    bid = B.exs_upload_ligands(batch, pocket_ids=[pid], stream=stream)
    torch.cuda.synchronize()
    upload_first_s = time.perf_counter() - t_up
    # the upload again, as a pipeline that keeps uploading sees it (the process's first call
    # also pays its first touch of host memory and its first threads): median of 3
    again = []
    for _ in range(3):
        t_up = time.perf_counter()
        b2 = B.exs_upload_ligands(batch, pocket_ids=[pid], stream=stream)
        torch.cuda.synchronize()
        again.append(time.perf_counter() - t_up)
        B.exs_release_ligands(b2)
    upload_s = float(np.median(again))
    unfold_ms = None
    if args.unfold_passes > 0:        # first step of the method, once per uploaded batch
        t_uf = time.perf_counter()
        B.exs_unfold_ligands(bid, s.torsion_steps, args.unfold_passes, stream=stream)
        unfold_ms = (time.perf_counter() - t_uf) * 1e3
        progress("unfolded %d ligands (%d passes): %.2f ms" % (batch.n_ligands, args.unfold_passes, unfold_ms))
    flags = B.EXS_FLAG_PERSISTENT if args.persistent else 0
    if args.rescore2 and args.rank_keep > 0:
        flags |= B.EXS_FLAG_RESCORE2
    prm = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, s.offset_step,
                          s.clash_cutoff, s.clash_penalty, top_k=0, poses_per_lane=args.ppl,
                          ligands_per_wg=args.lpw, flags=flags, cluster_rmsd_A=args.cluster_rmsd,
                          rank_keep=args.rank_keep)
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
    kms = float(np.mean(kernel_ms))
    traffic = measured_traffic(L) if (args.workload == "scale" and storage == 0 and args.ppl in (0, 1)
                                      and args.lpw in (0, 1) and not args.persistent) else None
    roof = roofline_of(B, batch, s, pocket.channels, kms, storage, traffic=traffic)
    probe = gather_probe(B, pid, storage, stream, batch, s, pocket.channels, kms)

    cpu = None
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        cpu = cpu_baseline(wl.name, pocket, batch, s)

    B.exs_release_ligands(bid)
    method_steps = None
    if args.workload == "scale" and not args.no_extra and args.ligands is None and storage == 0:
        progress("method steps: unfold, dock, rank, rescore (3,000 ligands)")
        method_steps = method_steps_leg(B, torch, S, pid, s, stream)
        progress("method steps: %s" % method_steps)
    B.exs_unload_pocket(pid)
    extra = None
    if args.workload == "scale" and not args.no_extra and args.ligands is None:
        extra = driver_legs(args, torch, S, B)
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
                            s.n_orient, s.torsion_steps, s.passes, s.n_offsets,
                            "one persistent launch" if args.persistent else "one launch per pocket"),
            "ligands": L, "atoms": A, "parallelism": "single GPU",
            "poses_per_lane": args.ppl, "ligands_per_wg": args.lpw,
            "rank_keep": args.rank_keep, "cluster_rmsd_A": args.cluster_rmsd if args.rank_keep else None,
            "rescore2": bool(args.rescore2 and args.rank_keep > 0),
            "unfold_passes": args.unfold_passes, "unfold_ms": None if unfold_ms is None else round(unfold_ms, 3),
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "gather_probe": probe,
        # not the value: the same steps with the host-side ligand upload (packing + PCIe) added
        "host_inclusive": {"upload_ms": round(upload_s * 1e3, 2),
                           "upload_first_ms": round(upload_first_s * 1e3, 2),
                           "docks_per_s": round(L / (upload_s + dt / args.steps), 2),
                           "docks_per_s_first": round(L / (upload_first_s + dt / args.steps), 2)},
        # identifies the results (runs with equal results print the same digest)
        "best_scores_sha256": __import__("hashlib").sha256(out["best_score"].tobytes()).hexdigest()[:16],
    }
    if method_steps is not None:
        line["method_steps"] = method_steps
    if extra is not None:
        legs = extra["legs"]
        line["batched"] = extra
        line["served"] = extra.pop("serving")
        line["campaign"] = extra.pop("campaign")
        pick = lambda d, *ks: {k: d[k] for k in ks if k in d}
        line["target"] = {
            "plain_f32_per_pocket": dict(pick(legs["plain_f32_per_pocket"], "docks_per_s"),
                                         **pick(legs["plain_f32_per_pocket"].get("vs_oracle", {}),
                                                "top1pct_overlap")),
            **{name: dict(pick(legs[name], "docks_per_s"),
                          roofline_frac=legs[name]["roofline"]["frac"],
                          **pick(legs[name].get("vs_oracle", {}), "top1pct_overlap"))
               for name in ("persistent_f32", "persistent_bf16_top8", "persistent_f16_top8")},
            "served_f32": pick(line["served"]["served_f32"], "docks_per_s", "p50_ms", "p99_ms"),
            "served_bf16_top8": pick(line["served"]["served_bf16_top8"], "docks_per_s", "p50_ms",
                                     "p99_ms"),
            "served_bf16_top8_own_load": pick(line["served"]["served_bf16_top8_own_load"],
                                              "docks_per_s", "p50_ms", "p99_ms",
                                              "offered_docks_per_s"),
            "plain_per_request_f32": pick(line["served"]["plain_per_request_f32"], "docks_per_s",
                                          "p50_ms", "p99_ms", "workers"),
            "campaign_f32": dict(pick(line["campaign"], "docks_per_s"),
                                 **pick(line["campaign"].get("vs_oracle", {}), "top1pct_overlap")),
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
