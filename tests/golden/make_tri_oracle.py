"""Write tri_oracle.json: the triharmonic oracle's fast tier (Sec. 4.2, "Triharmonic equation")
on the workload of Table 5 -- u = sin(k1 x) cos(k2 y) sin(k3 z) on the unit cube, clamped at
x = 0, Navier elsewhere -- at 32^3 and 64^3 for both (k1, k2, k3) settings, solved to a
relative Schur residual of 1e-13.  Stored per case: the max-norm error against the exact
solution, max |U|, and U at 512 seeded nodes ((z, y, x) indices of the nodal array) plus
64 on each of the four interior layers next to the clamped face (where the q-rows read U).
Calls only oracle/ and workloads/; about two minutes.

    python tests/golden/make_tri_oracle.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import triharmonic as T  # noqa: E402


def nodes(n, seed):
    rng = np.random.default_rng(seed)
    pts = [rng.integers(0, n + 1, size=(512, 3))]
    for layer in (1, 2, 3, 4):
        c = rng.integers(1, n, size=(64, 3))
        c[:, 2] = layer  # x index (memory order z, y, x): next to the clamped face x = 0
        pts.append(c)
    return np.concatenate(pts).astype(int)


def main():
    out = {"_cite": "Sec. 4.2 (Triharmonic equation), the workload of Table 5, solved by the oracle's "
                    "matrix-free tier (three sine-transform Poisson solves per Schur matvec, GMRES)",
           "cases": {}}
    for i, (n, k) in enumerate(((32, (5.0, 1.0, 5.0)), (32, (25.0, 5.0, 25.0)),
                                (64, (5.0, 1.0, 5.0)), (64, (25.0, 5.0, 25.0)))):
        t = time.time()
        p = W.example3_tri(n, k)
        U, Q, info = T.TriFast(p, workers=os.cpu_count()).solve(tol=1e-13)
        assert info["converged"], info["relres"]
        nd = nodes(n, 200 + i)
        err = float(np.abs(U - p.u_exact).max())
        key = f"{n}:" + ",".join(f"{v:g}" for v in k)
        out["cases"][key] = {"n": n, "k": list(k), "gmres_iters": info["iters"], "err_u_inf": err,
                             "u_max": float(np.abs(U).max()), "nodes": nd.tolist(),
                             "u": [float(U[c, b, a]) for c, b, a in nd]}
        print(f"{key}: err {err:.6e}, {info['iters']} iterations, {time.time() - t:.0f} s", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tri_oracle.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
