"""Serving (continuous batching) on the GPU through the C ABI: every request's
result equals the result of docking its ligands alone; invalid requests fail
alone; a small arena forces queueing (backpressure) without losing requests."""
import sys
import threading
import time

import numpy as np
import pytest

import exs_synth as S

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2110_11644_amd import binding
    binding.lib()
    return binding


WL = S.Workload("serve-test", 92, 0, 3, (32, 40, 48), 0.375, 8, ("lognormal", 35.0, 0.4, 10, 90),
                ("uniform", 0, 15), S.SearchSettings(64, 8, 1, 27))


@pytest.fixture(scope="module")
def setup(B):
    pockets = [S.make_pocket(WL, i) for i in range(3)]
    pids = [B.exs_load_pocket_grid(p.values, p.spacing, p.origin) for p in pockets]
    rng = np.random.default_rng(3)
    reqs = []
    start = 0
    for r in range(12):
        size = int(rng.integers(1, 24))
        ligs = S.make_ligands(WL, start, size)
        pk = int(rng.integers(0, 3))
        for l in ligs:
            l.pocket = pk
        reqs.append(S.batch_from_ligands(ligs))
        start += size
    yield pids, reqs
    for pid in pids:
        B.exs_unload_pocket(pid)


def params(B, s=WL.search):
    return B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, ligands_per_wg=1)


def alone(B, pids, batch):
    bid = B.exs_upload_ligands(batch, pocket_ids=pids)
    job = B.exs_dock_batch(bid, params(B))
    out = B.exs_get_best_poses(job, batch.n_ligands, int(batch.atom_offset[-1]))
    B.exs_release_job(job)
    B.exs_release_ligands(bid)
    return out


def serve(B, pids, reqs, gap_s=0.0, **cfg):
    srv = B.exs_server_create(pids, params(B), **cfg)
    results = {}
    try:
        ids = []
        for r in reqs:
            ids.append(B.exs_server_submit(srv, r, pocket_ids=pids))
            if gap_s:
                time.sleep(gap_s)
        for i, (rid, r) in enumerate(zip(ids, reqs)):
            results[i] = B.exs_server_poll(srv, rid, r.n_ligands, int(r.atom_offset[-1]))
        stats = B.exs_server_get_stats(srv)
    finally:
        B.exs_server_destroy(srv)
    return results, stats


def test_each_request_alone_equals_in_the_mix(B, setup):
    pids, reqs = setup
    log("serving: 12 requests, arrivals 2 ms apart")
    res, stats = serve(B, pids, reqs, gap_s=0.002)
    log("stats", stats)
    assert stats["completed"] == len(reqs)
    for i, r in enumerate(reqs):
        a = alone(B, pids, r)
        m = res[i]
        assert np.array_equal(a["best_score"], m["best_score"]), i
        assert np.array_equal(a["desc"]["orient"], m["desc"]["orient"]), i
        assert np.array_equal(a["desc"]["theta"], m["desc"]["theta"]), i
        assert np.array_equal(a["desc"]["tau"], m["desc"]["tau"]), i
        assert np.array_equal(a["coords"], m["coords"]), i
        assert m["latency_ms"] > 0


def test_small_arena_queues_requests_without_losing_any(B, setup):
    pids, reqs = setup
    log("serving: arena of 24 ligands, max 16 ligands per launch, one launch in flight")
    res, stats = serve(B, pids, reqs, max_arena_ligands=24, max_iter_ligands=16,
                       max_inflight_iters=1)
    log("stats", stats)
    assert stats["arena_ligands"] == 24
    assert stats["completed"] == len(reqs)
    assert stats["iterations"] >= sum(r.n_ligands for r in reqs) // 16
    ref, _ = serve(B, pids, reqs)
    for i in range(len(reqs)):
        assert np.array_equal(ref[i]["best_score"], res[i]["best_score"])


def test_invalid_request_fails_alone(B, setup):
    pids, reqs = setup
    srv = B.exs_server_create(pids, params(B))
    try:
        good = B.exs_server_submit(srv, reqs[0], pocket_ids=pids)
        bad = reqs[1].subset(range(reqs[1].n_ligands))
        bad.type[0] = 9                                  # channel out of range
        with pytest.raises(B.ExsError) as ei:
            B.exs_server_submit(srv, bad, pocket_ids=pids)
        assert ei.value.code == B.EXS_EINVAL
        with pytest.raises(B.ExsError) as ei:            # pocket the server does not hold
            B.exs_server_submit(srv, reqs[2], pocket_ids=[p + 100 for p in pids])
        assert ei.value.code == B.EXS_EINVAL
        good2 = B.exs_server_submit(srv, reqs[3], pocket_ids=pids)
        for rid, r in ((good, reqs[0]), (good2, reqs[3])):
            out = B.exs_server_poll(srv, rid, r.n_ligands, int(r.atom_offset[-1]))
            assert np.all(np.isfinite(out["best_score"]))
    finally:
        B.exs_server_destroy(srv)


def test_request_larger_than_the_arena_is_refused(B, setup):
    pids, reqs = setup
    srv = B.exs_server_create(pids, params(B), max_arena_ligands=4)
    try:
        big = max(reqs, key=lambda r: r.n_ligands)
        with pytest.raises(B.ExsError) as ei:
            B.exs_server_submit(srv, big, pocket_ids=pids)
        assert ei.value.code == B.EXS_ENOMEM
    finally:
        B.exs_server_destroy(srv)


def test_concurrent_submitters_equal_one_batch(B, setup):
    """A campaign-style stream: chunks submitted from three host threads at once (each packs
    its chunk) give, ligand for ligand, the results of one batch docked in a single launch."""
    pids, _ = setup
    ligs = S.make_ligands(WL, 500, 240)
    rng = np.random.default_rng(9)
    for l in ligs:
        l.pocket = int(rng.integers(0, 3))
    whole = S.batch_from_ligands(ligs)
    ref = alone(B, pids, whole)
    chunks = [S.batch_from_ligands(ligs[a:a + 30]) for a in range(0, len(ligs), 30)]
    srv = B.exs_server_create(pids, params(B))
    try:
        ids = [None] * len(chunks)
        nxt = [0]
        lock = threading.Lock()

        def packer():
            while True:
                with lock:
                    i = nxt[0]
                    nxt[0] += 1
                if i >= len(chunks):
                    return
                ids[i] = B.exs_server_submit(srv, chunks[i], pocket_ids=pids)
        th = [threading.Thread(target=packer) for _ in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        got = [B.exs_server_poll(srv, ids[i], c.n_ligands, int(c.atom_offset[-1]))
               for i, c in enumerate(chunks)]
    finally:
        B.exs_server_destroy(srv)
    best = np.concatenate([g["best_score"] for g in got])
    desc = np.concatenate([g["desc"] for g in got])
    xyz = np.concatenate([g["coords"] for g in got])
    assert np.array_equal(best, ref["best_score"])
    assert np.array_equal(desc["orient"], ref["desc"]["orient"])
    assert np.array_equal(desc["theta"], ref["desc"]["theta"])
    assert np.array_equal(xyz, ref["coords"])


def test_large_iterations_with_pocket_major_queues(B, setup):
    """Iterations large enough for the pocket-major work queues (each pocket of the iteration
    holds more ligands than the device has in flight: 3,072 one-wave ligands at 64
    orientations) give, ligand for ligand, the results of one plain launch."""
    pids, _ = setup
    ligs = S.make_ligands(WL, 2000, 7000)
    for i, l in enumerate(ligs):
        l.pocket = i % 2
    whole = S.batch_from_ligands(ligs)
    ref = alone(B, pids, whole)
    log("serving: one request of 7,000 ligands over 2 pockets, iterations of up to 8,192")
    res, stats = serve(B, pids, [whole], max_iter_ligands=8192)
    assert stats["completed"] == 1
    best, desc, xyz = res[0]["best_score"], res[0]["desc"], res[0]["coords"]
    assert np.array_equal(best, ref["best_score"])
    assert np.array_equal(desc["orient"], ref["desc"]["orient"])
    assert np.array_equal(desc["theta"], ref["desc"]["theta"])
    assert np.array_equal(desc["tau"], ref["desc"]["tau"])
    assert np.array_equal(xyz, ref["coords"])


def test_served_results_match_oracle(B, oracle_lib, setup):
    """Every ligand of three served requests (FP32 texels) against the FP64 oracle: the served
    best pose passes the best-pose acceptance (score of its descriptor, best within tolerance
    or a near tie, coordinates within 0.01 A)."""
    from parity import check_best_pose
    O = oracle_lib
    pids, reqs = setup
    grids = [O.Grid.of(S.make_pocket(WL, i)) for i in range(3)]
    prm = O.Params.of(WL.search)
    res, _ = serve(B, pids, reqs[:3], gap_s=0.002)
    n = 0
    for i, r in enumerate(reqs[:3]):
        for l in range(r.n_ligands):
            lig = r.ligand(l)
            a0, a1 = int(r.atom_offset[l]), int(r.atom_offset[l + 1])
            check_best_pose(O, grids[lig.pocket], prm, lig, res[i]["best_score"][l],
                            res[i]["desc"][l], res[i]["coords"][a0:a1])
            n += 1
    log("served ligands checked against the oracle:", n)


def test_served_16bit_topk_matches_oracle(B, oracle_lib):
    """The mixed-precision served form: BF16 pockets, top-8 FP64 rescoring.  Per ligand of three
    requests: the served FP64 score is the oracle's FP64 score of the served descriptor on the
    FP32 master, the coordinates are that pose, and the FP64 best equals the oracle's own run
    of the same path (search on the rounded grid, its top 8 rescored on the master) within the
    FP32 tolerance unless that selection is a near tie."""
    from parity import gpu_desc_to_theta_tau, oracle_topk_fp64_best, tol
    O = oracle_lib
    pockets = [S.make_pocket(WL, i) for i in range(3)]
    pids = [B.exs_load_pocket_grid(p.values, p.spacing, p.origin, 1) for p in pockets]
    s = WL.search
    prm_gpu = B.search_params(s.n_orient, s.torsion_steps, s.passes, s.n_offsets, top_k=8,
                              ligands_per_wg=1)
    rng = np.random.default_rng(31)
    reqs = []
    for r in range(3):
        ligs = S.make_ligands(WL, 3000 + 20 * r, int(rng.integers(4, 12)))
        for l in ligs:
            l.pocket = r
        reqs.append(S.batch_from_ligands(ligs))
    srv = B.exs_server_create(pids, prm_gpu)
    try:
        ids = [B.exs_server_submit(srv, r, pocket_ids=pids) for r in reqs]
        res = [B.exs_server_poll(srv, h, r.n_ligands, int(r.atom_offset[-1]))
               for h, r in zip(ids, reqs)]
    finally:
        B.exs_server_destroy(srv)
        for pid in pids:
            B.exs_unload_pocket(pid)
    g32 = [O.Grid.of(p) for p in pockets]
    g16 = [O.Grid(S.to_bf16_rne(p.values), p.spacing, p.origin) for p in pockets]
    prm = O.Params.of(s)
    n_amb = 0
    for r, out in zip(reqs, res):
        for l in range(r.n_ligands):
            lig = r.ligand(l)
            d = out["desc"][l]
            th, ta = gpu_desc_to_theta_tau(d, len(lig.rot))
            e, _, amb, X = O.rescore_desc(g32[lig.pocket], prm, lig, int(d["orient"]), th, ta)
            assert abs(float(d["score_fp64"]) - e) <= 1e-9 * max(1.0, abs(e)) + amb
            assert float(out["best_score"][l]) == np.float32(d["score_fp64"])
            a0, a1 = int(r.atom_offset[l]), int(r.atom_offset[l + 1])
            assert np.max(np.abs(out["coords"][a0:a1] - X)) < 1e-5
            b64, k64, ambiguous = oracle_topk_fp64_best(O, g16[lig.pocket], g32[lig.pocket], prm,
                                                        lig, 8)
            if abs(float(d["score_fp64"]) - b64) > tol(b64):
                assert ambiguous, "ligand %d: served fp64 best %.9g (k=%d) vs oracle %.9g (k=%d)" % (
                    l, d["score_fp64"], d["orient"], b64, k64)
                n_amb += 1
    log("served 16-bit ligands:", sum(r.n_ligands for r in reqs), "accepted on a near tie:", n_amb)


def request_bytes(r, K, top_k=0):
    """Device bytes a request holds while admitted (the formula exs.h states)."""
    return (r.n_ligands * (76 + 12 * K + 28 * top_k) + 68 * int(r.atom_offset[-1])
            + int(r.rot_offset[-1]) * (21 + K + top_k))


def test_byte_budget_holds_requests_back(B, setup):
    """A server whose HBM budget leaves room for about two requests' bytes beyond its iteration
    scratch: with all 12 requests submitted at once, some wait for admission (backpressure),
    the admitted bytes never exceed the budget, and every result equals the unconstrained
    server's.  The default budget is clamped to the device's free memory."""
    import torch
    pids, reqs = setup
    srv = B.exs_server_create(pids, params(B))
    st = B.exs_server_get_stats(srv)
    B.exs_server_destroy(srv)
    free, total = torch.cuda.mem_get_info()
    assert 0 < st["budget_bytes"] <= free
    scratch = st["budget_bytes"] - st["arena_budget_bytes"]
    big = max(request_bytes(r, WL.search.n_orient) for r in reqs)
    budget = scratch + 2 * big + big // 2
    log("budget %d B: iteration scratch %d B + %d B for requests (largest %d B)" % (
        budget, scratch, budget - scratch, big))
    res, stats = serve(B, pids, reqs, hbm_budget_bytes=budget)
    log("stats", stats)
    assert stats["budget_bytes"] == budget and stats["arena_budget_bytes"] == budget - scratch
    assert stats["completed"] == len(reqs)
    assert stats["peak_queued"] >= 1
    assert 0 < stats["peak_admitted_bytes"] <= budget - scratch
    assert stats["admitted_bytes"] == 0
    ref, _ = serve(B, pids, reqs)
    for i in range(len(reqs)):
        assert np.array_equal(ref[i]["best_score"], res[i]["best_score"])
        assert np.array_equal(ref[i]["coords"], res[i]["coords"])
    with pytest.raises(B.ExsError) as ei:        # a request larger than the byte budget
        srv = B.exs_server_create(pids, params(B), hbm_budget_bytes=scratch + big // 2)
        try:
            B.exs_server_submit(srv, max(reqs, key=lambda r: request_bytes(r, 64)), pocket_ids=pids)
        finally:
            B.exs_server_destroy(srv)
    assert ei.value.code == B.EXS_ENOMEM


def test_overlapping_iterations_equal_one_at_a_time(B, setup):
    """Small iterations, two in flight on their own hardware queues (the search writes each
    ligand's result straight into the iteration's pinned buffer), give bit for bit the results
    of the same requests served one iteration at a time."""
    pids, reqs = setup
    log("serving: 12 requests, iterations of 16 ligands, 2 in flight vs 1")
    two, st2 = serve(B, pids, reqs, max_iter_ligands=16, max_inflight_iters=2)
    one, st1 = serve(B, pids, reqs, max_iter_ligands=16, max_inflight_iters=1)
    log("stats", st2, st1)
    assert st2["iterations"] >= 2 and st1["iterations"] >= 2
    for i in range(len(reqs)):
        for key in ("best_score", "coords"):
            assert np.array_equal(two[i][key], one[i][key]), (i, key)
        for key in ("orient", "theta", "tau"):
            assert np.array_equal(two[i]["desc"][key], one[i]["desc"][key]), (i, key)
