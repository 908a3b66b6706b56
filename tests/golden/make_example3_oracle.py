"""Write example3_oracle.json: the oracle's direct solve of the 3-D oscillatory example of
Sec. 4.1 (Table 3, u = sin(k1 x) cos(k2 y) sin(k3 z)) at 32^3.

Variable alpha = x^2 + y^2 + z^2 + 1 and beta = x + y + z + 10, clamped at x = 0 and Navier
elsewhere, inhomogeneous boundary data, for the two (k1, k2, k3) settings of Table 3.
Stored per setting: the max-norm error against the exact solution and U at 64 seeded
interior nodes ((z, y, x) indices of the nodal array).  Calls only oracle/ and workloads/; several minutes per setting (sparse LU).

    python tests/golden/make_example3_oracle.py
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
    out = {"_cite": "Sec. 4.1, the 3-D oscillatory example (the workload of Table 3) at 32^3, solved by the "
                    "oracle's direct tier",
           "n": N, "nodes": None, "cases": {}}
    nodes = np.random.default_rng(47).integers(1, N, size=(64, 3))
    out["nodes"] = nodes.tolist()
    for k in ((5.0, 1.0, 5.0), (25.0, 5.0, 25.0)):
        t = time.time()
        pr = W.example3(N, k)
        U, V, Q, asm = direct.solve(pr)
        err = float(np.abs(U - pr.u_exact).max())
        key = ",".join(f"{v:g}" for v in k)
        out["cases"][key] = {"err_u_inf": err, "u": [float(U[c, b, a]) for c, b, a in nodes]}
        print(f"k = ({key}): err {err:.6e}, {time.time() - t:.0f} s", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "example3_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
