"""Write the 127-qubit golden runs of the FP64 oracle (tests/golden/eagle_chi*_theta*.json).

Calls only the oracle (oracle/bp_tns.py) and the seeded lattice generator.  Each file holds one
whole run of the kicked Ising circuit on the 127-qubit heavy-hex lattice (Fig. 1; Eq.
"Propagator"), with truncation to chi active from the step where the bonds saturate: <Z_v> after
every step, the BP sweeps, the summed discarded weight and, per step, the bond dimension of every
edge and the cut diagnostics (smallest relative gap of a chi-limited cut, number of
near-degenerate cuts).  The GPU parity tests compare their runs with these values.

Usage: python tests/golden/make_eagle_goldens.py CHI THETA [DEPTH]
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import bp_tns as O  # noqa: E402
from paper_2306_14887_amd import lattice as L  # noqa: E402


def golden_path(chi: int, theta: float) -> str:
    return os.path.join(HERE, f"eagle_chi{chi}_theta{theta:.6f}.json")


def main() -> None:
    chi, theta = int(sys.argv[1]), float(sys.argv[2])
    depth = int(sys.argv[3]) if len(sys.argv) > 3 else 20
    lat = L.eagle()
    opt = O.Options(chi=chi)
    t0 = time.time()
    res = O.solve(lat.n_sites, lat.edges, lat.colour, theta, depth, opt)
    out = {
        "workload": "127-qubit heavy-hex lattice, kicked Ising, BP-gauged simple update",
        "generator": "tests/golden/make_eagle_goldens.py (FP64 oracle)",
        "n_sites": lat.n_sites, "edges": lat.edges.tolist(), "colour": lat.colour.tolist(),
        "chi": chi, "theta": theta, "depth": depth,
        "bp_tol": opt.bp_tol, "bp_max_iter": opt.bp_max_iter,
        "svd_cutoff": opt.svd_cutoff, "eig_cutoff": opt.eig_cutoff,
        "z": [[float(x) for x in row] for row in res.z],
        "bp_iters": [int(x) for x in res.bp_iters],
        "bp_residual": [float(x) for x in res.bp_residual],
        "discarded": [float(x) for x in res.discarded],
        "bond_dims": res.bond_dims.tolist(),
        "min_cut_gap": [None if math.isinf(g) else float(g) for g in res.min_cut_gap],
        "degenerate_cuts": [int(x) for x in res.degenerate_cuts],
        "oracle_seconds": time.time() - t0,
    }
    with open(golden_path(chi, theta), "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")
    print(f"chi={chi} theta={theta:.6f}: {out['oracle_seconds']:.0f} s, "
          f"sweeps {sum(out['bp_iters'])}, degenerate cuts {sum(out['degenerate_cuts'])}")


if __name__ == "__main__":
    main()
