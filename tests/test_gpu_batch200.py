"""The batched workload at its configured size against stored FP64 oracle
results: all 64 uneven 2-D slices (sides 48..256, P in {30, 60}, Q in {100,
400, 1600}) solved together in shared launches for the configured 200
iterations, in bf16x3 (the workload's precision) and float32; six slices (per
Q the smallest and the largest) compared with tests/golden/batch200_c4.npz,
written by tests/golden/make_batch200_golden.py from the generator and oracle/
only. Compared per slice: the full Q-vectors of z^200 at its sampled voxels,
every voxel's spectral sum and norm, every node's spatial sum and ||z^200||;
relative errors (the form of Eq. DFCS) within 1e-5 (float32) and 1e-3
(bf16x3), the worst sampled voxel within ten times that.
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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_configured_batch_against_stored_oracle(torch_cuda, prec):
    torch = torch_cuda
    g = np.load(os.path.join(HERE, "golden", "batch200_c4.npz"))
    probs = synth.generate_batch()
    iters = int(g["iters"])
    assert len(probs) == int(g["nslices"])
    say("configured batch", prec, len(probs), "slices,", sum(p.N for p in probs), "voxels,", iters, "iters")
    tol = TOL[prec]
    with _ffi.BatchMapper([p.K for p in probs], [p.grid for p in probs]) as bm:
        Ms = [torch.tensor(p.m, dtype=torch.float32, device="cuda") for p in probs]
        Fs = bm.solve_torch(Ms, [p.lam for p in probs], [p.beta for p in probs], iters, precision=prec)
        torch.cuda.synchronize()
        st = bm.stats()
        assert st["njobs"] == len(probs) and st["solo_jobs"] == 0
        for k in (int(v) for v in g["slices"]):
            F = Fs[k]
            idx = torch.as_tensor(g[f"s{k}_index"], device="cuda")
            z_s = F[idx].double().cpu().numpy()
            errs = {
                "sampled": rel(z_s, g[f"s{k}_z"]),
                "worst voxel": max(rel(z_s[i], g[f"s{k}_z"][i]) for i in range(len(z_s))),
                "spectral sums": rel(F.double().sum(dim=1).cpu().numpy(), g[f"s{k}_z_sum_q"]),
                "voxel norms": rel(F.double().norm(dim=1).cpu().numpy(), g[f"s{k}_z_norm_q"]),
                "spatial sums": rel(F.double().sum(dim=0).cpu().numpy(), g[f"s{k}_z_sum_n"]),
                "||z||": abs(float(F.double().norm()) - float(g[f"s{k}_norm_z"])) / float(g[f"s{k}_norm_z"]),
            }
            say(f"  slice {k} {probs[k].grid} Q {probs[k].Q}:",
                ", ".join(f"{n} {v:.2e}" for n, v in errs.items()))
            for n, v in errs.items():
                assert v <= (10 * tol if n == "worst voxel" else tol), (k, n, v)
