"""Write tests/golden/iters<K>_<case>.npz: FP64 oracle results of whole
problems at their configured iteration count K.

Calls only the seeded generator (inputs) and oracle/ (values); rank and xi_p
come from the oracle's own rules (Sec. III-F, Eq. sigma_cond). Cases:

* c2crop: the c2 recipe (3-D diffusion-relaxation, P = 60, Q = 1600, seed 2)
  drawn on a 128 x 128 x 8 grid -- 256 bricks of 16 x 8 x 4, the float32
  launch shape of the 128 x 128 x 64 workload -- 300 iterations;
* c3: the c3 recipe (fingerprinting-like, P = 1000, Q = 1024, seed 3) at its
  full 96 x 96 x 32 size, 300 iterations;
* c1: the c1 recipe (2-D diffusion-relaxation, P = 30, Q = 100) at its full
  32 x 32 size, 500 iterations (brick boundaries of its 16 x 2 x 1 split).

Stored per case: the sampled voxels (grid corners, voxels on each face and
edge, both sides of brick boundaries in x, y and z, random voxels) with the
full Q-vectors of z^K, f^K and d^K there; for every voxel the spectral
sum of z^K and ||z_n^K||; for every node the spatial sum of z^K; the
Frobenius norms of z, f and d; the objective of Eq. (spat) at z^K; rank,
xi_p, lambda, beta.

    python tests/golden/make_iters300_golden.py [case ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2401_12890_amd import synth  # noqa: E402

CASES = {
    "c2crop": dict(recipe="c2", grid=(128, 128, 8), brick=(16, 8, 4), iters=300),
    "c3": dict(recipe="c3", grid=None, brick=(16, 4, 4), iters=300),
    "c1": dict(recipe="c1", grid=None, brick=(16, 2, 1), iters=500),
}


def file_name(case):
    return f"iters{CASES[case]['iters']}_{case}.npz"


def sample_voxels(grid, brick, n_random=24, seed=11):
    """Grid corners, face and edge voxels, voxels on both sides of brick
    boundaries, and seeded random voxels (duplicates removed, order kept)."""
    nx, ny, nz = grid
    bx, by, bz = brick
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = []
    for x in (0, nx - 1):
        for y in (0, ny - 1):
            for z in (0, nz - 1):
                pts.append((x, y, z))
    # one voxel inside each face and on each edge
    pts += [(0, ny // 3, nz // 2), (nx - 1, 2 * ny // 3, nz // 3), (nx // 3, 0, nz // 2),
            (2 * nx // 3, ny - 1, nz // 2), (nx // 2, ny // 3, 0), (nx // 3, ny // 2, nz - 1),
            (nx // 2, 0, 0), (0, ny // 2, nz - 1), (nx - 1, ny - 1, nz // 2)]
    # both sides of brick boundaries (x, y, z and their corners)
    for k in range(1, 4):
        x = min(k * bx, nx - 1)
        y = min(k * by, ny - 1)
        z = min(k * bz, nz - 1)
        pts += [(x - 1, y - 1, z - 1), (x, y, z), (x - 1, y, z), (x, y - 1, z), (x, y, z - 1),
                (x - 1, ny // 2, nz // 2), (nx // 2, y - 1, nz // 2), (nx // 2, ny // 2, z - 1)]
    for _ in range(n_random):
        pts.append(tuple(int(rng.integers(0, s)) for s in (nx, ny, nz)))
    seen, out = set(), []
    for p in pts:
        p = tuple(int(v) for v in p)
        if p not in seen and all(0 <= p[i] < grid[i] for i in range(3)):
            seen.add(p)
            out.append(p)
    return out


def run(case):
    spec = CASES[case]
    prob = synth.generate(spec["recipe"], grid=spec["grid"])
    nx, ny, nz = prob.grid
    t0 = time.time()
    iters = spec["iters"]
    out = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, iters)
    U, s, V = oracle.thin_svd(prob.K)
    rank = oracle.rank_rule(s, 0)
    xi = oracle.xi_rule(prob.lam, prob.grid)
    assert out["rank"] == rank and out["xi"] == xi
    z, f, d = out["z"], out["f"], out["d"]
    J = oracle.objective(out["K_r"], prob.m, z, prob.grid, prob.lam)
    pts = sample_voxels(prob.grid, spec["brick"])
    idx = np.asarray([x + nx * (y + ny * zz) for (x, y, zz) in pts], dtype=np.int64)
    path = os.path.join(HERE, file_name(case))
    np.savez_compressed(
        path, recipe=spec["recipe"], grid=np.asarray(prob.grid, dtype=np.int64),
        iters=iters, rank=rank, xi_p=xi, lam=prob.lam, beta=prob.beta, objective=J,
        voxels=np.asarray(pts, dtype=np.int64), index=idx,
        z=z[idx], f=f[idx], d=d[idx],
        z_sum_q=z.sum(axis=1), z_norm_q=np.sqrt((z * z).sum(axis=1)), z_sum_n=z.sum(axis=0),
        norm_z=np.linalg.norm(z), norm_f=np.linalg.norm(f), norm_d=np.linalg.norm(d))
    print(f"{case}: grid {prob.grid} {iters} iterations rank {rank} xi {xi:.6g} J {J:.10g} "
          f"samples {len(pts)} ({time.time() - t0:.0f} s)", flush=True)


def main(argv):
    for case in (argv or list(CASES)):
        run(case)


if __name__ == "__main__":
    main(sys.argv[1:])
