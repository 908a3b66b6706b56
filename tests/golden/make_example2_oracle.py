"""Write example2_oracle.json: the oracle's direct solve of Example 2 (Sec. 4.1) at 32^3.

Variable alpha = x^2 + y^2 + z^2 + 1 and beta = x + y + z + 10, clamped at x = 0 and Navier
elsewhere, for the two (q, p) settings of Table 2.  Stored per setting: the max-norm error
against the exact solution and U at 64 seeded interior nodes ((z, y, x) indices of the nodal
array).  Calls only oracle/ and workloads/; several minutes per setting (sparse LU).

    python tests/golden/make_example2_oracle.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import direct  # noqa: E402

N = 32


def main():
    out = {"_cite": "Sec. 4.1, Example 2 (the workload of Table 2) at 32^3, solved by the oracle's direct tier",
           "n": N, "nodes": None, "cases": {}}
    nodes = np.random.default_rng(43).integers(1, N, size=(64, 3))
    out["nodes"] = nodes.tolist()
    for q, p in ((10.0, 0.2), (5.0, 1.0)):
        t = time.time()
        pr = W.example2(N, q, p)
        U, V, Q, asm = direct.solve(pr)
        err = float(np.abs(U - pr.u_exact).max())
        out["cases"][f"{q:g},{p:g}"] = {"err_u_inf": err, "u": [float(U[k, j, i]) for k, j, i in nodes]}
        print(f"(q, p) = ({q:g}, {p:g}): err {err:.6e}, {time.time() - t:.0f} s", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "example2_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
