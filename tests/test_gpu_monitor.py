"""GPU monitoring against the FP64 oracle's history, through the C ABI.

At every check the device reports, in float64: the objective of Eq. (spat)
with R of Eq. (l2) at z^k, the dual residual beta ||z^k - z^{k-1}||, ||z^k||,
the primal residual ||z^k - f^k|| of the splitting f = z (opt-in), and the
distance from a converged solution (Eq. DFCS) of z^k and of f^k against a
reference map f* set on the context. The oracle's history (Algorithm 2 run
step by step, its own objective and norms) is the reference; tolerances are
1e-9 relative in float64 and 1e-4 in float32 (primal residual: 1e-4 of itself
plus 1e-5 of ||z||, since it is a difference of two nearly equal maps).
"""
import numpy as np
import pytest

import oracle
from paper_2401_12890_amd import _ffi, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


CASES = [("c1", (24, 20, 1), "fp64", "fused"), ("c1", (24, 20, 1), "fp64", "unfused"),
         ("c2", (18, 14, 5), "fp32", "fused"), ("c3", (12, 10, 4), "bf16x3", "fused"),
         ("c2", (11, 9, 3), "fp32", "unfused")]
TOL = {"fp64": 1e-9, "fp32": 1e-4, "bf16x3": 1e-3}


@pytest.mark.parametrize("recipe,grid,prec,kernel", CASES,
                         ids=[f"{c[0]}-{c[2]}-{c[3]}" for c in CASES])
def test_monitor_history_matches_oracle(torch_cuda, recipe, grid, prec, kernel):
    iters, every = 60, 10
    prob = synth.generate(recipe, grid=grid, iters=iters)
    # a converged reference: the unapproximated K, many iterations (Eq. DFCS)
    f_star = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, 1500, rank=-1)["z"]
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, iters, track_every=every,
                       f_star=f_star)
    say("monitor", recipe, grid, prec, kernel, "rank", ref["rank"])
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        mp.set_reference(f_star)
        z = mp.solve(prob.m, prob.lam, prob.beta, iters, precision=prec, kernel=kernel,
                     check_every=every, primal=True)
        st = mp.stats()
        z_plain = mp.solve(prob.m, prob.lam, prob.beta, iters, precision=prec, kernel=kernel)
    assert np.array_equal(z, z_plain)          # monitoring does not touch the iterates
    tol = TOL[prec]
    J = {k: v for (k, v, _) in ref["hist"]}
    D = {k: v for (k, _, v) in ref["hist"]}
    Pr = {k: v for (k, v, _) in ref["hist_f"]}
    Df = {k: v for (k, _, v) in ref["hist_f"]}
    assert st["hist_iter"] == list(range(every, iters + 1, every))
    for i, k in enumerate(st["hist_iter"]):
        zk = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, k)["z"]
        zk1 = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, k - 1)["z"]
        zn = np.linalg.norm(zk)
        assert st["hist_objective"][i] == pytest.approx(J[k], rel=tol), k
        assert st["hist_dfcs"][i] == pytest.approx(D[k], rel=tol), k
        assert st["hist_dfcs_f"][i] == pytest.approx(Df[k], rel=tol), k
        assert st["hist_znorm"][i] == pytest.approx(zn, rel=tol), k
        dual = prob.beta * np.linalg.norm(zk - zk1)
        assert abs(st["hist_dual"][i] - dual) <= tol * dual + (0 if prec == "fp64" else 1e-5 * prob.beta * zn), k
        assert abs(st["hist_primal"][i] - Pr[k]) <= tol * Pr[k] + (0 if prec == "fp64" else 1e-5 * zn), k


def test_monitor_without_reference_or_primal(torch_cuda):
    prob = synth.generate("c2", grid=(13, 11, 3), iters=20)
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, 20, track_every=5)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        mp.solve(prob.m, prob.lam, prob.beta, 20, precision="fp32", check_every=5)
        st = mp.stats()
    assert st["hist_primal"] == [-1.0] * 4 and st["hist_dfcs"] == [-1.0] * 4
    J = {k: v for (k, v, _) in ref["hist"]}
    for k, v in zip(st["hist_iter"], st["hist_objective"]):
        assert v == pytest.approx(J[k], rel=1e-4)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_gemm_path_monitoring(torch_cuda, prec):
    """The exact-rank GEMM path (voxel-major state) reports the same history."""
    iters, every = 30, 10
    prob = synth.generate("c2", grid=(14, 10, 3), iters=iters)       # P = 60: rank 60 > 32
    f_star = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, 800, rank=-1)["z"]
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, iters, rank=-1,
                       track_every=every, f_star=f_star)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        mp.set_reference(f_star)
        z = mp.solve(prob.m, prob.lam, prob.beta, iters, precision=prec, rank=-1, kernel="gemm",
                     check_every=every)
        st = mp.stats()
    assert st["kernel"] == 3
    tol = TOL[prec] if prec == "bf16x3" else 1e-4
    J = {k: v for (k, v, _) in ref["hist"]}
    D = {k: v for (k, _, v) in ref["hist"]}
    for i, k in enumerate(st["hist_iter"]):
        assert st["hist_objective"][i] == pytest.approx(J[k], rel=tol), k
        assert st["hist_dfcs"][i] == pytest.approx(D[k], rel=tol), k
    assert np.linalg.norm(z - ref["z"]) <= 1e-5 * np.linalg.norm(ref["z"]) * (100 if prec == "bf16x3" else 1)


def test_reference_errors(torch_cuda):
    prob = synth.random_problem(6, 5, (3, 2, 1), seed=3)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        bad = np.zeros((prob.N, prob.Q))
        with pytest.raises(_ffi.SsmapError) as e:
            mp.set_reference(bad)
        assert e.value.status == _ffi.SSMAP_EINVAL
        bad[0, 0] = np.nan
        with pytest.raises(_ffi.SsmapError) as e:
            mp.set_reference(bad)
        assert e.value.status == _ffi.SSMAP_ENONFINITE
        with pytest.raises(_ffi.SsmapError) as e:     # no f on the GEMM path
            mp.solve(prob.m, 0.1, 1.0, 5, precision="fp32", kernel="gemm", check_every=1,
                     primal=True)
        assert e.value.status == _ffi.SSMAP_EINVAL
        mp.set_reference(None)
        z = mp.solve(prob.m, 0.1, 1.0, 5, check_every=5, primal=True)
        assert np.isfinite(z).all() and mp.stats()["hist_dfcs"] == [-1.0]
