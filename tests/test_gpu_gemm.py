"""Exact-rank GEMM path against the FP64 oracle, through the C ABI.

Ranks above 32 (up to min(P, Q), the unapproximated dictionary) run the two
contractions as MFMA-tiled GEMMs over all voxels; the result must match the
oracle at the same rank to the precision's tolerance.
"""
import numpy as np
import pytest

import oracle
from paper_2401_12890_amd import _ffi, synth

pytestmark = pytest.mark.gpu

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


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    # recipe, grid, rank, iters  (rank -1: min(P, Q))
    ("c3", (10, 9, 4), -1, 20),       # r = 1000: Qg = Rg = 1024
    ("c2", (11, 7, 5), -1, 30),       # r = 60, Q = 1600: Qg = 1664, Rg = 128
    ("c2", (13, 6, 1), 45, 25),       # planar, rank 45
    ("c1", (17, 11, 1), -1, 40),      # r = 30 < 32 through the GEMM path too
]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("recipe,grid,rank,iters", CASES)
def test_gemm_path_matches_oracle(torch_cuda, recipe, grid, rank, iters, prec):
    p = synth.generate(recipe, grid=grid, iters=iters)
    ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, iters, rank=rank)
    with _ffi.Mapper(p.K, p.grid) as mp:
        F = mp.solve(p.m, p.lam, p.beta, iters, precision=prec, rank=rank, kernel="gemm")
        st = mp.stats()
    err = relerr(F, ref["z"])
    say(recipe, grid, "rank", ref["rank"], prec, err, "gemm ms", st["gemm_ms"])
    assert st["kernel"] == 3 and st["rank"] == ref["rank"]
    assert st["gemm_ms"] > 0
    Qg = (p.Q + 127) // 128 * 128
    Rg = (ref["rank"] + 127) // 128 * 128
    assert st["gemm_flops"] == 4.0 * Qg * Rg * (3 if prec == "bf16x3" else 1) * p.N * iters
    assert err <= TOL[prec], (recipe, grid, prec, err)


def test_auto_takes_the_gemm_path_above_rank_32(torch_cuda):
    p = synth.generate("c2", grid=(9, 8, 3), iters=10)
    with _ffi.Mapper(p.K, p.grid) as mp:
        mp.solve(p.m, p.lam, p.beta, 10, precision="fp32", rank=40)
        assert mp.stats()["kernel"] == 3
        # monitoring runs on the GEMM path too; the primal residual needs f,
        # which only the unfused path forms
        mp.solve(p.m, p.lam, p.beta, 10, precision="fp32", rank=40, check_every=5)
        assert mp.stats()["kernel"] == 3
        mp.solve(p.m, p.lam, p.beta, 10, precision="fp32", rank=40, check_every=5, primal=True)
        assert mp.stats()["kernel"] == 1
        mp.solve(p.m, p.lam, p.beta, 10, precision="fp32", rank=40, keep_aux=True)
        assert mp.stats()["kernel"] == 3
        mp.solve(p.m, p.lam, p.beta, 10, precision="fp32")
        assert mp.stats()["kernel"] == 2


def test_gemm_path_with_a_mask(torch_cuda):
    p = synth.generate("c2", grid=(12, 10, 4), iters=20)
    nx, ny, nz = p.grid
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    mask = (((x - 6) / 5.0) ** 2 + ((y - 5) / 4.0) ** 2 + ((z - 1.5) / 2.0) ** 2 <= 1.0).reshape(-1)
    ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 20, rank=-1, mask=mask)
    with _ffi.Mapper(p.K, p.grid) as mp:
        mp.set_mask(mask)
        F = mp.solve(p.m, p.lam, p.beta, 20, precision="fp32", rank=-1, kernel="gemm")
    assert np.all(F[~mask] == 0.0)
    assert relerr(F, ref["z"]) <= TOL["fp32"]


def test_gemm_path_rejections(torch_cuda):
    p = synth.generate("c1", grid=(6, 5, 1))
    with _ffi.Mapper(p.K, p.grid) as mp:
        for kw in (dict(precision="fp64"), dict(precision="fp32", check_every=5, primal=True)):
            with pytest.raises(_ffi.SsmapError) as e:
                mp.solve(p.m, p.lam, p.beta, 5, kernel="gemm", **kw)
            assert e.value.status == _ffi.SSMAP_EINVAL, kw


AUX_CASES = [("c3", (10, 9, 4), -1, 20), ("c2", (13, 6, 1), 45, 25), ("c2", (9, 8, 3), 40, 1)]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("recipe,grid,rank,iters", AUX_CASES)
def test_gemm_path_aux_output(torch_cuda, recipe, grid, rank, iters, prec):
    """f^K and d^K from the library path's bracket (Algorithm 2's f- and d-steps
    from z^k, u^k = V_r w^k and z^{k+1}) against the oracle at ten times the
    tolerance, d's denominator floored at beta ||z|| as elsewhere."""
    p = synth.generate(recipe, grid=grid, iters=iters)
    ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, iters, rank=rank)
    with _ffi.Mapper(p.K, p.grid) as mp:
        F = mp.solve(p.m, p.lam, p.beta, iters, precision=prec, rank=rank, kernel="gemm", keep_aux=True)
        st = mp.stats()
        f, d = mp.aux()
    floor = p.beta * np.linalg.norm(ref["z"])
    ef, ed = relerr(f, ref["f"]), np.linalg.norm(d - ref["d"]) / max(np.linalg.norm(ref["d"]), floor)
    say(recipe, grid, "rank", ref["rank"], prec, "z", relerr(F, ref["z"]), "f", ef, "d", ed)
    assert st["kernel"] == 3 and st["gemm_library"] == 1
    assert relerr(F, ref["z"]) <= TOL[prec]
    assert ef <= 10 * TOL[prec] and ed <= 10 * TOL[prec]
