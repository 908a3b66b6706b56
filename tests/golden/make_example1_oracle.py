"""Write example1_oracle.json: the oracle's solution of Example 1 (Sec. 4.1) at 4096 x 4096.

The direct tier cannot factor this size, so the fast tier (Algorithm 1 with library sine
transforms, itself pinned to the direct tier) solves it to a Schur residual of 1e-13.  Stored
per eps: the max-norm error against the exact solution and U at 64 seeded interior nodes
(row-major (y, x) indices of the nodal array).  Calls only oracle/ and workloads/; takes
several minutes per eps on one core.

    python tests/golden/make_example1_oracle.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import fast  # noqa: E402

N = 4096


def main():
    out = {"_cite": "Sec. 4.1, Example 1 (the workload of Table 1) at N = 4096, solved by the oracle's fast "
                    "tier to ||b - S Q|| / ||b|| <= 1e-13",
           "n": N, "nodes": None, "eps": {}}
    rng = np.random.default_rng(41)
    nodes = rng.integers(1, N, size=(64, 2))
    out["nodes"] = nodes.tolist()
    for eps in ("1e-4", "1e-5"):
        t = time.time()
        p = W.example1(N, float(eps))
        U, V, Q, info = fast.FastTier(p, workers=4).solve(tol=1e-13, restart=60)
        assert info["converged"], info
        err = float(np.abs(U - p.u_exact).max())
        out["eps"][eps] = {"err_u_inf": err, "u": [float(U[j, i]) for j, i in nodes],
                           "gmres_iters": int(info["iters"])}
        print(f"eps {eps}: err {err:.6e}, {info['iters']} iterations, {time.time() - t:.0f} s", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "example1_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
