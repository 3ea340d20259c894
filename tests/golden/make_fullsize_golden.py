"""Write tests/golden/fullsize_<workload>.json: oracle values at sampled voxels
of the full-size workloads after 4 iterations (c2 and c3 at the rank of the
rank rule, c3x: the c3 recipe at the unapproximated rank min(P, Q) = 1000).

Calls only the seeded generator (inputs) and oracle/ (values). For each
sampled voxel the FP64 oracle is run on a crop of half-width 5 around it
(z^4 at a voxel depends only on data within 3 voxels, so the crop gives the
full-grid value there). Stored per voxel: its coordinates, ||z^4|| and the
projection <z^4, g> on a fixed seeded Gaussian vector g (PCG64 seed 2401),
which lets the benchmark check its own full-size output without the oracle.

    python tests/golden/make_fullsize_golden.py [workload ...]
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2401_12890_amd import synth  # noqa: E402

ITERS = 4
PROJ_SEED = 2401
# workload -> (recipe, rank parameter of the rank rule: 0 the 0.005 % rule, -1 min(P, Q))
WORKLOADS = {"c2": ("c2", 0), "c3": ("c3", 0), "c3x": ("c3", -1)}


def points(grid, n=12, seed=7):
    nx, ny, nz = grid
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, 0, nz // 2), (nx // 2, ny // 2, 0),
           (15, 8, 4), (16, 7, 3)]
    pts += [tuple(int(rng.integers(0, s)) for s in (nx, ny, nz)) for _ in range(n - len(pts))]
    return pts


def main(argv):
    for name in (argv or list(WORKLOADS)):
        recipe, rank_param = WORKLOADS[name]
        prob = synth.generate(recipe)
        U, s, V = oracle.thin_svd(prob.K)
        rank = oracle.rank_rule(s, rank_param)
        xi = oracle.xi_rule(prob.lam, prob.grid)
        g = np.random.Generator(np.random.PCG64(PROJ_SEED)).standard_normal(prob.Q)
        nx, ny, nz = prob.grid
        h = ITERS + 1
        rec = {"workload": name, "grid": list(prob.grid), "iters": ITERS, "rank": int(rank),
               "xi_p": xi, "lambda": prob.lam, "beta": prob.beta, "projection_seed": PROJ_SEED,
               "samples": []}
        for (x, y, z) in points(prob.grid):
            x0, x1 = max(0, x - h), min(nx, x + h + 1)
            y0, y1 = max(0, y - h), min(ny, y + h + 1)
            z0, z1 = max(0, z - h), min(nz, z + h + 1)
            idx = [xx + nx * (yy + ny * zz) for zz in range(z0, z1) for yy in range(y0, y1)
                   for xx in range(x0, x1)]
            sub = oracle.ladmm(prob.K, prob.m[idx], (x1 - x0, y1 - y0, z1 - z0), prob.lam,
                               prob.beta, ITERS, rank=rank, xi=xi)
            c = (x - x0) + (x1 - x0) * ((y - y0) + (y1 - y0) * (z - z0))
            zr = sub["z"][c]
            rec["samples"].append({"voxel": [x, y, z], "norm": float(np.linalg.norm(zr)),
                                   "proj": float(zr @ g)})
        with open(os.path.join(HERE, f"fullsize_{name}.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        print(name, "rank", rank, "samples", len(rec["samples"]))


if __name__ == "__main__":
    main(sys.argv[1:])
