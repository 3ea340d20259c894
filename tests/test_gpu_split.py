"""The chunk-split kernel (one workgroup per brick and 16-node chunk, the rank
vectors carried as per-chunk partial products) against the FP64 oracle,
through the C ABI: relative error of z^K (the form of Eq. DFCS) within 1e-10 in
float64 and 1e-5 in float32, the monitored objective within 1e-9 / 1e-4.
"""
import numpy as np
import pytest

import oracle
from paper_2401_12890_amd import _ffi, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


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


@pytest.mark.parametrize("rank", [0, -1])
def test_c1_full_size_takes_the_split_kernel(torch_cuda, rank):
    prob = synth.generate("c1")
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, prob.iters, rank=rank,
                       track_every=100)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        z = mp.solve(prob.m, prob.lam, prob.beta, prob.iters, precision="fp64", rank=rank,
                     check_every=100)
        st = mp.stats()
        z2 = mp.solve(prob.m, prob.lam, prob.beta, prob.iters, precision="fp64", rank=rank)
    say("c1 split rank", st["rank"], "err", relerr(z, ref["z"]))
    assert st["kernel"] == 4
    assert np.array_equal(z, z2)                  # chunk partials are added in a fixed order
    assert relerr(z, ref["z"]) <= TOL["fp64"]
    J = {k: v for (k, v, _) in ref["hist"]}
    for k, v in zip(st["hist_iter"], st["hist_objective"]):
        assert v == pytest.approx(J[k], rel=1e-9)


# (recipe, grid, spectral grid side, precision, iterations): planar and volumetric
# bricks, ragged in every axis, ranks on both sides of 16 and in the float32
# tail bucket (17..20)
CASES = [("c1", (21, 13, 1), 10, "fp64", 40), ("c1", (18, 10, 6), 10, "fp64", 30),
         ("c2", (37, 11, 1), 20, "fp32", 40), ("c2", (19, 9, 5), 12, "fp32", 40),
         ("c2", (23, 17, 3), 20, "fp32", 30), ("c1", (30, 22, 1), 6, "fp32", 40)]


@pytest.mark.parametrize("recipe,grid,n,prec,iters", CASES,
                         ids=[f"{c[0]}-{'x'.join(map(str, c[1]))}-{c[3]}" for c in CASES])
def test_split_parity(torch_cuda, recipe, grid, n, prec, iters):
    prob = synth.generate(recipe, grid=grid, iters=iters, overrides=dict(n1=n, n2=n))
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, iters, track_every=iters)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        z = mp.solve(prob.m, prob.lam, prob.beta, iters, precision=prec, kernel="split",
                     check_every=iters)
        st = mp.stats()
        zf = mp.solve(prob.m, prob.lam, prob.beta, iters, precision=prec, kernel="fused")
    say("split", recipe, grid, prec, "Q", prob.Q, "rank", st["rank"], "err", relerr(z, ref["z"]))
    assert st["kernel"] == 4 and st["rank"] == ref["rank"]
    assert relerr(z, ref["z"]) <= TOL[prec]
    assert relerr(z, zf) <= TOL[prec]
    J_tol = 1e-9 if prec == "fp64" else 1e-4
    assert st["hist_objective"][-1] == pytest.approx(ref["hist"][-1][1], rel=J_tol)


def test_split_with_a_mask(torch_cuda):
    prob = synth.generate("c1", grid=(29, 23, 1), iters=30)
    yy, xx = np.mgrid[0:23, 0:29]
    mask = ((xx - 14) ** 2 + (yy - 11) ** 2 < 100) & ~((xx - 16) ** 2 + (yy - 12) ** 2 < 6)
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, 30, mask=mask.reshape(-1))
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        mp.set_mask(mask.reshape(-1))
        z = mp.solve(prob.m, prob.lam, prob.beta, 30, precision="fp64", kernel="split")
    assert np.all(z[~mask.reshape(-1)] == 0.0)
    assert relerr(z, ref["z"]) <= TOL["fp64"]


def test_split_rejections(torch_cuda):
    prob = synth.generate("c1", grid=(8, 8, 1), iters=5)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        for kw in (dict(precision="bf16x3"), dict(keep_aux=True), dict(check_every=1, primal=True)):
            with pytest.raises(_ffi.SsmapError) as e:
                mp.solve(prob.m, prob.lam, prob.beta, 5, kernel="split", **kw)
            assert e.value.status == _ffi.SSMAP_EINVAL, kw
        # AUTO with aux output keeps the fused kernel
        mp.solve(prob.m, prob.lam, prob.beta, 5, keep_aux=True)
        assert mp.stats()["kernel"] == 2
