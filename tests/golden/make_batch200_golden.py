"""Write tests/golden/batch200_c4.npz: FP64 oracle results for slices of the
batched workload (64 uneven 2-D slices, sides 48..256, P in {30, 60}, Q in
{100, 400, 1600}, seeded) at its configured 200 iterations.

Calls only the seeded generator (inputs) and oracle/ (values); rank and xi_p
come from the oracle's own rules (Sec. III-F, Eq. sigma_cond). The slices are,
for each Q, the smallest and the largest of the batch (six in all); each is
solved alone by Algorithm 2 (a batch job's iterates are those of its own
problem). Stored per slice k (keys s<k>_...): the sampled voxels (corners,
edge and brick-boundary voxels, random voxels) with the full Q-vector of z^200
there; for every voxel the spectral sum and the norm of z^200; for every node
the spatial sum; ||z^200||; rank and xi_p.

    python tests/golden/make_batch200_golden.py
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


def chosen_slices(probs):
    """For each Q: the slices with the fewest and the most voxels."""
    byq = {}
    for p in probs:
        byq.setdefault(p.Q, []).append(p)
    out = []
    for q in sorted(byq):
        lst = sorted(byq[q], key=lambda p: (p.N, p.meta["slice"]))
        out += [lst[0], lst[-1]]
    return out


def sample_voxels(grid, n_random=32, seed=17):
    """Corners, voxels on each edge, both sides of 16-voxel brick boundaries in x
    and of 8-voxel ones in y, and seeded random voxels (distinct, order kept)."""
    nx, ny, _ = grid
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1),
           (nx // 2, 0), (nx // 3, ny - 1), (0, ny // 2), (nx - 1, ny // 3)]
    for k in (1, 2, 5):
        x, y = min(16 * k, nx - 1), min(8 * k, ny - 1)
        pts += [(x - 1, y - 1), (x, y), (x - 1, y), (x, y - 1)]
    while len(pts) < 16 + 12 + n_random:
        pts.append((int(rng.integers(nx)), int(rng.integers(ny))))
    seen, idx = set(), []
    for x, y in pts:
        n = x + nx * y
        if n not in seen:
            seen.add(n)
            idx.append(n)
    return np.array(idx, dtype=np.int64)


def main():
    probs = synth.generate_batch()
    iters = probs[0].iters
    out = {"iters": np.int64(iters), "nslices": np.int64(len(probs))}
    slices = []
    for p in chosen_slices(probs):
        k = p.meta["slice"]
        t0 = time.time()
        ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, iters)
        z = ref["z"]
        idx = sample_voxels(p.grid)
        out[f"s{k}_index"] = idx
        out[f"s{k}_z"] = z[idx]
        out[f"s{k}_z_sum_q"] = z.sum(axis=1)
        out[f"s{k}_z_norm_q"] = np.linalg.norm(z, axis=1)
        out[f"s{k}_z_sum_n"] = z.sum(axis=0)
        out[f"s{k}_norm_z"] = np.float64(np.linalg.norm(z))
        out[f"s{k}_rank"] = np.int64(ref["rank"])
        out[f"s{k}_xi_p"] = np.float64(ref["xi"])
        slices.append(k)
        print(f"slice {k}: grid {p.grid} P {p.P} Q {p.Q} rank {ref['rank']} ||z|| "
              f"{np.linalg.norm(z):.10g} ({time.time() - t0:.0f} s)", flush=True)
    out["slices"] = np.array(slices, dtype=np.int64)
    np.savez_compressed(os.path.join(HERE, "batch200_c4.npz"), **out)


if __name__ == "__main__":
    main()
