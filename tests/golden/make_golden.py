"""Writes oracle_small.json: a regression fixture of the FP64 oracle.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import exs_synth as S  # noqa: E402
import oracle as O     # noqa: E402


def main():
    O.build()
    g = O.Grid.of(S.make_pocket("small"))
    prm = O.Params.of(S.SMALL.search)
    out = {"_source": "FP64 oracle, small workload (48^3 x 4 grid, 64 orientations, 16 torsion "
                      "steps, 1 pass), ligands 0 and 1", "ligands": []}
    for idx in (0, 1):
        lig = S.make_ligands("small", idx, 1)[0]
        r = O.dock_ligand(g, prm, lig)
        out["ligands"].append({"index": idx, "best_k": r["best_k"],
                               "score": [float(v) for v in r["score"]],
                               "theta": r["theta"].tolist()})
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
