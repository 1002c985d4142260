"""Writes fault_6912x10752_L15_cost.json: the optimal total integer flow cost
of the 6912 x 10752 strike-slip fault scene (L = 15, 3 % nodata, seed 2),
computed by the CPU oracle alone (residues, FP64 cost table, edge costs, one
path at a time successive shortest paths with a binary heap).

Single-threaded; the shortest-path phase takes hours on one host core.
Usage: python tests/golden/make_fault_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def main():
    import numpy as np
    import oracle
    from paper_2609_36267_amd import synth

    t0 = time.time()
    sc = synth.config("c2")
    m, n = sc.psi.shape
    print(f"scene {m}x{n} generated in {time.time() - t0:.1f} s", flush=True)
    T = oracle.build_lut(sc.looks)
    res, _, ground = oracle.residues(sc.psi, sc.valid)
    costs, cst = oracle.edge_costs(sc.psi, sc.coh, sc.valid, T, want_stats=True)
    print(f"residues {int(np.abs(res).sum())} ground {ground} costs {cst}", flush=True)
    t1 = time.time()
    (dkx, dky, pot, total), ms = oracle.mcf(res, costs, m=m, n=n, want_stats=True)
    dt = time.time() - t1
    cert = oracle.check_optimal(res, costs, dkx, dky, pot)
    assert cert["ok"], cert
    out = {
        "scene": "strike-slip fault 6912x10752, L=15, 3% nodata, seed 2 (synth.config('c2'))",
        "total_cost": int(total),
        "residues": int(np.abs(res).sum()),
        "ground_charge": int(ground),
        "valid_edges": int(cst["valid_edges"]),
        "steep_zeroed": int(cst["steep_zeroed"]),
        "nonzero_dk": int(np.count_nonzero(dkx) + np.count_nonzero(dky)),
        "oracle_mcf_seconds": round(dt, 1),
        "certificate": "reduced costs >= 0 and divergence = residues (oracle check_optimal)",
    }
    with open(os.path.join(HERE, "fault_6912x10752_L15_cost.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
