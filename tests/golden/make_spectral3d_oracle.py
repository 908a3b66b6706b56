"""Write spectral3d_oracle.json: the oracle's fast tier (Algorithm 1 with library sine
transforms, pinned to the direct coupled solve) on 3-D grids whose every axis length has a
length-specialised transform on the GPU (32, 64, 96, 128), i.e. the grids the GPU solves
through its spectral lift and face sums (the benchmarked path).

Cases (all with the variable alpha of the 3-D benchmark configuration, alpha = 1 + 0.5 sin(2 pi
x) sin(2 pi y) sin(2 pi z), and u = sin^2(pi x) sin^2(pi y) sin^2(pi z), fully clamped):
  c3_64        the unit cube at 64^3
  c3_32x64x96  the box [0,1] x [0,1.3] x [0,0.8] on 32 x 64 x 96 intervals (unequal axes
               and spacings; inhomogeneous data on the faces y = 1.3, z = 0.8)
  c3_128       the unit cube at 128^3
Each is solved with GMRES(30) to a relative Schur residual of 1e-14 (1e-15 where it gets
there).  Stored per case: the max-norm error against the exact solution, max |U|, and U at
seeded nodes ((z, y, x) indices of the nodal array): 1024 spread over the grid and 64 on each
of the three interior layers next to each face (where the lift and the boundary gather act).
Calls only oracle/ and workloads/; a few minutes in all.

    python tests/golden/make_spectral3d_oracle.py
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

CASES = {
    "c3_64": ((64, 64, 64), (1.0, 1.0, 1.0), 1e-15),
    "c3_32x64x96": ((32, 64, 96), (1.0, 1.3, 0.8), 1e-14),
    "c3_128": ((128, 128, 128), (1.0, 1.0, 1.0), 1e-14),
}


def sample_nodes(n, seed):
    """(z, y, x) nodal indices: spread over the whole grid, plus the layers 1..3 next to
    every face."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    pts = [np.stack([rng.integers(0, nz + 1, 1024), rng.integers(0, ny + 1, 1024),
                     rng.integers(0, nx + 1, 1024)], axis=1)]
    for axis in range(3):
        for side in (0, 1):
            for layer in (1, 2, 3):
                c = np.stack([rng.integers(1, nz, 64), rng.integers(1, ny, 64), rng.integers(1, nx, 64)], axis=1)
                col = 2 - axis  # memory order (z, y, x)
                c[:, col] = layer if side == 0 else n[axis] - layer
                pts.append(c)
    return np.concatenate(pts).astype(int)


def main():
    out = {"_cite": "Sec. 2.3 Lemma 1 and Algorithm 1 (the oracle's fast tier, itself pinned to the direct "
                    "solve of the coupled system eq-coupled) on grids solved through the GPU's spectral path",
           "cases": {}}
    for i, (name, (n, hi, tol)) in enumerate(CASES.items()):
        t = time.time()
        p = W.manufactured(W.C3_ALPHA, W.C3_U, n, (0.0, 0.0, 0.0), hi)
        ft = fast.FastTier(p)
        U, V, Q, info = ft.solve(tol=tol, max_iters=600)
        assert info["converged"], (name, info["relres"])
        nodes = sample_nodes(n, 100 + i)
        err = float(np.abs(U - p.u_exact).max())
        out["cases"][name] = {
            "n": list(n), "hi": list(hi), "tol": tol, "gmres_iters": info["iters"],
            "relres": float(info["relres"]), "err_u_inf": err, "u_max": float(np.abs(U).max()),
            "nodes": nodes.tolist(), "u": [float(U[c, b, a]) for c, b, a in nodes],
        }
        print(f"{name}: {info['iters']} iterations, relres {info['relres']:.2e}, err {err:.6e}, "
              f"{time.time() - t:.0f} s", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "spectral3d_oracle.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
