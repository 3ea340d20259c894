"""The allocation-free entry point (ssmap_solve_device_noalloc) against the
allocating one (ssmap_solve_device), through the C ABI.

Every device buffer of an allocation-free solve comes from one static array
per GPU, which keeps the previous call's contents. Each case runs two calls in
a row on the same array, the second on a smaller problem, so leftovers of the
first call would show up in the second; both must equal the allocating entry
point's maps bit for bit (same kernels, same arithmetic order). A problem above
the array's size is refused with EINVAL before any device work, and the
context stays usable.
"""
import numpy as np
import pytest

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


# (recipe, overrides, precision, larger grid, smaller grid, iterations, check_every)
CASES = [
    ("c1", {}, "fp64", (32, 32, 1), (12, 10, 1), 60, 0),
    ("c2", dict(n1=20, n2=20), "fp32", (40, 36, 6), (20, 14, 3), 30, 10),
    ("c3", {}, "bf16x3", (24, 20, 4), (10, 8, 3), 30, 0),
    ("c2", dict(n1=10, n2=10), "fp32", (50, 30, 4), (9, 7, 2), 20, 0),
]


@pytest.mark.parametrize("recipe,over,prec,big,small,iters,check", CASES,
                         ids=[f"{c[0]}-{c[2]}" for c in CASES])
def test_noalloc_equals_device_entry(torch_cuda, recipe, over, prec, big, small, iters, check):
    torch = torch_cuda
    dt = torch.float64 if prec == "fp64" else torch.float32
    for grid in (big, small):
        prob = synth.generate(recipe, grid=grid, iters=iters, overrides=over)
        say("noalloc", recipe, prec, grid, "Q", prob.Q)
        M = torch.tensor(prob.m, dtype=dt, device="cuda")
        with _ffi.Mapper(prob.K, prob.grid) as ref_mp:
            F_ref = ref_mp.solve_torch(M, prob.lam, prob.beta, iters, precision=prec,
                                       check_every=check)
            torch.cuda.synchronize()
            st_ref = ref_mp.stats()
        with _ffi.Mapper(prob.K, prob.grid) as mp:
            F = torch.full_like(F_ref, float("nan"))
            mp.solve_torch(M, prob.lam, prob.beta, iters, F=F, precision=prec, check_every=check,
                           noalloc=True)
            torch.cuda.synchronize()
            st = mp.stats()
        assert st["kernel"] == st_ref["kernel"]
        assert 0 < st["device_bytes"] <= _ffi.NOALLOC_MAX_BYTES
        assert torch.equal(F, F_ref), float((F - F_ref).abs().max())
        if check:
            assert st["hist_objective"] == st_ref["hist_objective"]
            assert st["hist_dual"] == st_ref["hist_dual"]


def test_noalloc_refuses_what_does_not_fit(torch_cuda):
    torch = torch_cuda
    prob = synth.generate("c2", grid=(64, 64, 8), iters=2)    # 2 x 1600 x 32768 x 4 B of state
    M = torch.tensor(prob.m, dtype=torch.float32, device="cuda")
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        with pytest.raises(_ffi.SsmapError) as e:
            mp.solve_torch(M, prob.lam, prob.beta, 2, precision="fp32", noalloc=True)
        assert e.value.status == _ffi.SSMAP_EINVAL
        with pytest.raises(_ffi.SsmapError) as e:
            mp.solve_torch(M, prob.lam, prob.beta, 2, precision="fp32", noalloc=True,
                           keep_aux=True)
        assert e.value.status == _ffi.SSMAP_EINVAL
        F = mp.solve_torch(M, prob.lam, prob.beta, 2, precision="fp32")   # still usable
        torch.cuda.synchronize()
        assert torch.isfinite(F).all()
