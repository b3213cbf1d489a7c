"""Writes oracle_batched_20k.npz: FP64 oracle best scores of a declared subset of the batched
workload, the reference of the precision comparison (top-1 % hit overlap against the oracle).

Subset: ligands 0 .. 19,999 of the batched workload (seeded counter-based streams, so they are
the same ligands the 100,000-ligand runs dock first), each against its own pocket of the 15,
K=256 orientations, S=32 torsion steps, 2 passes, 27 rigid offsets of 0.5 A, FP32 master grids.
Top 1 % of the subset = 200 hits.

Calls only the oracle and the seeded input generators (chunks of 500 ligands, OpenMP over the
ligands of a chunk; a partial file lets an interrupted run resume).  Run from the repository
root:  python tests/golden/make_oracle_batched.py [--threads N] [--count N]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np     # noqa: E402

import exs_synth as S  # noqa: E402
import oracle as O     # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "oracle_batched_20k.npz")
CHUNK = 500


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--count", type=int, default=20000)
    args = ap.parse_args()
    O.build()
    wl = S.BATCHED
    grids = [O.Grid.of(S.make_pocket(wl, i)) for i in range(wl.n_pockets)]
    prm = O.Params.of(wl.search)
    n = args.count
    part = OUT + ".partial.npz"
    best = np.full(n, np.nan)
    best_k = np.full(n, -1, np.int32)
    near_best = np.zeros(n, bool)
    n_near = np.zeros(n, np.int32)
    done = 0
    if os.path.exists(part):
        z = np.load(part)
        done = int(z["done"])
        best[:done], best_k[:done] = z["best_score"][:done], z["best_k"][:done]
        near_best[:done], n_near[:done] = z["near_tie_best"][:done], z["near_tie_count"][:done]
    t0 = time.perf_counter()
    while done < n:
        m = min(CHUNK, n - done)
        batch = S.make_ligand_batch(wl, done, m)
        r = O.dock_batch(grids, prm, batch, threads=args.threads, per_orientation=True)
        best[done:done + m] = r["best_score"]
        best_k[done:done + m] = r["best_k"]
        near_best[done:done + m] = r["near_tie"][np.arange(m), r["best_k"]]
        n_near[done:done + m] = r["near_tie"].sum(axis=1)
        done += m
        np.savez(part, done=done, best_score=best, best_k=best_k, near_tie_best=near_best,
                 near_tie_count=n_near)
        print("%d / %d ligands, %.0f s" % (done, n, time.perf_counter() - t0), flush=True)
    meta = {"source": "FP64 oracle (oracle/exs_oracle.c), batched workload ligands 0..%d, each "
                      "against its own pocket; K=%d, S=%d, P=%d, T=%d, offset step %.3f A, clash "
                      "cutoff %.3f A, penalty %.3f; FP32 master grids" % (
                          n - 1, prm.n_orient, prm.torsion_steps, prm.passes, prm.n_offsets,
                          prm.offset_step, prm.clash_cutoff, prm.clash_penalty),
            "seed": S.SEED, "workload": wl.name, "count": n,
            "near_tie": "orientation flagged by the oracle (a decision gap below 1e-4 relative, "
                        "clash pairs within 1e-4 A of the cutoff counted either way)"}
    np.savez_compressed(OUT, best_score=best, best_k=best_k, near_tie_best=near_best,
                        near_tie_count=n_near, meta=np.array(json.dumps(meta)))
    os.remove(part)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
