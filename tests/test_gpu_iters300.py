"""The 3-D workloads at their configured 300 iterations against stored FP64
oracle results (tests/golden/iters300_<case>.npz, written by
tests/golden/make_iters300_golden.py, which calls only the generator and
oracle/):

* c2crop: the c2 recipe (P = 60, Q = 1600, seed 2) on a 128 x 128 x 8 grid,
  256 bricks of 16 x 8 x 4 -- the float32 launch shape of the 128 x 128 x 64
  workload;
* c3: the c3 recipe (P = 1000, Q = 1024, bf16x3) at its full 96 x 96 x 32.

Both run with the library's own rank and xi_p rules, asserted equal to the
oracle's. Compared: the full Q-vectors of z^300, f^300 and d^300 at 64 sampled
voxels (grid corners, faces and edges, both sides of brick boundaries, random
voxels); over every voxel, the spectral sum and the norm of z^300; over every
node, the spatial sum of z^300; the Frobenius norms of z, f and d; and the
objective of Eq. (spat) at z^300. Relative errors (the form of Eq. DFCS) are
bounded by 1e-5 (float32) and 1e-3 (bf16x3) for z and its sums, ten times that
for f and d (d's denominator floored at beta ||z||), and 1e-4 for the
objective.
"""
import os

import numpy as np
import pytest

from paper_2401_12890_amd import _ffi, synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"fp32": 1e-5, "bf16x3": 1e-3}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def rel(a, b, floor=0.0):
    nb = max(float(np.linalg.norm(b)), floor)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b))) / nb


@pytest.mark.parametrize("case", ["c2crop", "c3"])
def test_iters300_against_stored_oracle(torch_cuda, case):
    torch = torch_cuda
    g = np.load(os.path.join(HERE, "golden", f"iters300_{case}.npz"))
    recipe = str(g["recipe"])
    grid = tuple(int(v) for v in g["grid"])
    prob = synth.generate(recipe, grid=grid)
    prec = prob.precision
    iters = int(g["iters"])
    tol = TOL[prec]
    say("iters300", case, grid, prec, iters)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        M = torch.tensor(prob.m, dtype=torch.float32, device="cuda")
        F = mp.solve_torch(M, prob.lam, prob.beta, iters, precision=prec, keep_aux=True,
                           check_every=iters)
        torch.cuda.synchronize()
        st = mp.stats()
        assert st["kernel"] == 2                   # the fused kernel of the workload's launch
        assert st["rank"] == int(g["rank"])
        assert st["xi_p"] == pytest.approx(float(g["xi_p"]), rel=1e-13)
        idx = torch.as_tensor(g["index"], device="cuda")
        z_s = F[idx].double().cpu().numpy()
        zsum_q = F.double().sum(dim=1).cpu().numpy()
        znorm_q = F.double().norm(dim=1).cpu().numpy()
        zsum_n = F.double().sum(dim=0).cpu().numpy()
        norm_z = float(F.double().norm())
        del M, F
        f, d = mp.aux()
    f_s, d_s = f[g["index"]], d[g["index"]]
    norm_f, norm_d = float(np.linalg.norm(f)), float(np.linalg.norm(d))
    del f, d
    beta_z = prob.beta * float(g["norm_z"])
    errs = {
        "z sampled": rel(z_s, g["z"]),
        "z per-voxel max": max(rel(z_s[i], g["z"][i]) for i in range(len(z_s))),
        "z spectral sums": rel(zsum_q, g["z_sum_q"]),
        "z voxel norms": rel(znorm_q, g["z_norm_q"]),
        "z spatial sums": rel(zsum_n, g["z_sum_n"]),
        "||z||": abs(norm_z - float(g["norm_z"])) / float(g["norm_z"]),
        "f sampled": rel(f_s, g["f"]),
        "d sampled": rel(d_s, g["d"], floor=prob.beta * float(np.linalg.norm(g["z"]))),
        "||f||": abs(norm_f - float(g["norm_f"])) / float(g["norm_f"]),
        "||d||": abs(norm_d - float(g["norm_d"])) / max(float(g["norm_d"]), beta_z),
        "objective": abs(st["hist_objective"][-1] - float(g["objective"])) / float(g["objective"]),
    }
    for k, v in errs.items():
        say(f"  {k}: {v:.3e}")
    for k in ("z sampled", "z spectral sums", "z voxel norms", "z spatial sums", "||z||"):
        assert errs[k] <= tol, (k, errs[k])
    assert errs["z per-voxel max"] <= 10 * tol, errs["z per-voxel max"]
    for k in ("f sampled", "d sampled", "||f||", "||d||"):
        assert errs[k] <= 10 * tol, (k, errs[k])
    assert errs["objective"] <= 1e-4, errs["objective"]
