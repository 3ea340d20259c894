"""GPU parity of libssmap against the FP64 oracle, through the C ABI.

Tolerances (relative Frobenius error over all N*Q entries, the form of
Eq. DFCS): 1e-10 for the float64 path, 1e-5 for float32, 1e-3 for the
bf16x3 split-precision path; the objective within 1e-4.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2401_12890_amd import _ffi, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-3}
DT = {"fp64": np.float64, "fp32": np.float32, "bf16x3": np.float32}


def relerr(a, b, floor=0.0):
    """||a - b|| / ||b|| (the DFCS form), with the denominator floored at
    `floor` for quantities that converge to zero (the dual d and the
    residual-like parts of f at an interior solution)."""
    nb = max(np.linalg.norm(b), floor)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def kernels_for(prec, r):
    """Kernel families that exist for a precision and rank."""
    return ["unfused", "fused"]


def run(mp, prob, prec, kernel, iters, ref=None, **kw):
    if ref is not None:
        kw.setdefault("xi_p", ref["xi"])
        kw.setdefault("rank", ref["rank"])
    try:
        return mp.solve(prob.m, prob.lam, prob.beta, iters, precision=prec, kernel=kernel, **kw)
    except _ffi.SsmapError as e:
        if kernel == "fused" and e.status == _ffi.SSMAP_EINVAL and "no fused kernel" in str(e):
            pytest.skip("no fused kernel for this precision/rank")
        raise


# ------------------------------------------------------------ setup (a0)
def test_singular_values_match_lapack(torch_cuda):
    for name, grid in (("c1", (4, 4, 1)), ("c2", (3, 3, 2)), ("c3", (2, 2, 2))):
        prob = synth.generate(name, grid=grid)
        say("svd", name)
        with _ffi.Mapper(prob.K, prob.grid) as mp:
            s = mp.singular_values()
        U, s_ref, V = oracle.thin_svd(prob.K)
        assert s.shape == s_ref.shape
        assert np.allclose(s, s_ref, rtol=1e-12, atol=1e-13 * s_ref[0])


def test_rank_and_xi_rules(torch_cuda):
    prob = synth.generate("c1")
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, 0)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        mp.solve(prob.m, prob.lam, prob.beta, 1, precision="fp64")
        st = mp.stats()
    assert st["rank"] == ref["rank"]
    assert st["xi_p"] == pytest.approx(ref["xi"], rel=1e-13)
    assert st["dtd_norm"] == pytest.approx(oracle.dtd_norm(prob.grid), rel=1e-13)


# ------------------------------------------------------------ config 1, full size
@pytest.mark.parametrize("kernel", ["unfused", "fused"])
@pytest.mark.parametrize("rank", [0, -1])
def test_c1_fp64_full(torch_cuda, kernel, rank):
    prob = synth.generate("c1")
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, prob.iters, rank=rank,
                       track_every=100)
    say("c1 fp64", kernel, "rank", ref["rank"])
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        z = run(mp, prob, "fp64", kernel, prob.iters, ref, keep_aux=True, check_every=100)
        f, d = mp.aux()
        st = mp.stats()
    assert st["rank"] == ref["rank"]
    assert relerr(z, ref["z"]) <= TOL["fp64"], relerr(z, ref["z"])
    assert relerr(f, ref["f"]) <= TOL["fp64"], relerr(f, ref["f"])
    assert relerr(d, ref["d"]) <= TOL["fp64"], relerr(d, ref["d"])
    assert z.min() >= 0.0
    # monitored objective at iterations 100..500 vs the oracle's objective
    J_ref = {k: J for (k, J, _) in ref["hist"]}
    for k, J in zip(st["hist_iter"], st["hist_objective"]):
        assert J == pytest.approx(J_ref[k], rel=1e-9)


# ------------------------------------------------------------ crops of configs 2 and 3
CROPS = [
    ("c2", (20, 18, 5), "fp32", 60),      # ragged in every axis, Q = 1600
    ("c2", (33, 7, 3), "bf16x3", 40),
    ("c3", (17, 9, 4), "bf16x3", 40),     # P = 1000, Q = 1024
    ("c3", (10, 6, 3), "fp32", 40),
    ("c2", (9, 11, 2), "fp64", 30),
]


@pytest.mark.parametrize("kernel", ["unfused", "fused"])
@pytest.mark.parametrize("name,grid,prec,iters", CROPS)
def test_crop_parity(torch_cuda, kernel, name, grid, prec, iters):
    prob = synth.generate(name, grid=grid, iters=iters)
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, iters, track_every=iters)
    say("crop", name, grid, prec, kernel, "rank", ref["rank"])
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        z = run(mp, prob, prec, kernel, iters, ref, keep_aux=True, check_every=iters)
        f, d = mp.aux()
        st = mp.stats()
    tol = TOL[prec]
    assert relerr(z, ref["z"]) <= tol, relerr(z, ref["z"])
    assert relerr(f, ref["f"]) <= 10 * tol, relerr(f, ref["f"])
    assert relerr(d, ref["d"]) <= 10 * tol, relerr(d, ref["d"])
    assert z.min() >= 0.0
    assert st["hist_objective"][-1] == pytest.approx(ref["hist"][-1][1], rel=1e-4)


# ------------------------------------------------------------ persistent brick walk
# Short spectra on the double-buffered bricks run a grid of one workgroup per
# CU, so with more bricks than CUs a workgroup takes several in turn and
# prefetches the next brick's first chunks. Float32 volumetric (16 x 8 x 4,
# Q = 36): 320 bricks, the table in eight contiguous XCD runs, and 350, plain
# round robin. Float64 planar (16 x 8 x 1, Q = 100): 312 bricks. Float32
# planar (16 x 16 x 1, Q = 36): 304 bricks. With Q = 16 each brick is a single
# chunk, so the stream moves on to the next brick at every chunk (324, 306 and
# 289 bricks, rank below 17). Ragged in every axis.
WALKS = [("c2", (60, 62, 38), "fp32", 6), ("c2", (76, 54, 38), "fp32", 6),
         ("c1", (200, 190, 1), "fp64", 10), ("c2", (300, 250, 1), "fp32", 6),
         ("c2", (64, 72, 36), "fp32", 4), ("c1", (260, 140, 1), "fp64", 4),
         ("c2", (270, 260, 1), "fp32", 4)]


@pytest.mark.parametrize("recipe,grid,prec,n", WALKS)
def test_persistent_walk_parity(torch_cuda, recipe, grid, prec, n):
    iters = 12
    prob = synth.generate(recipe, grid=grid, iters=iters, overrides=dict(n1=n, n2=n))
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, iters, track_every=iters)
    say("walk", recipe, grid, prec, "rank", ref["rank"])
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        z = run(mp, prob, prec, "fused", iters, ref, keep_aux=True, check_every=iters)
        f, d = mp.aux()
        st = mp.stats()
    tol = TOL[prec]
    assert relerr(z, ref["z"]) <= tol, relerr(z, ref["z"])
    assert relerr(f, ref["f"]) <= 10 * tol, relerr(f, ref["f"])
    assert relerr(d, ref["d"]) <= 10 * tol, relerr(d, ref["d"])
    assert z.min() >= 0.0
    assert st["hist_objective"][-1] == pytest.approx(ref["hist"][-1][1], rel=1e-4)


# ------------------------------------------------------------ float64 volumetric bricks
# float64 3-D grids take 16 x 4 x 2 double-buffered bricks when 16 x 4 x 4 would
# not fill the CUs, else 16 x 4 x 4: one grid on each side of the rule.
@pytest.mark.parametrize("grid", [(40, 28, 24), (64, 64, 20)])
def test_fp64_volumetric_bricks(torch_cuda, grid):
    iters = 12
    prob = synth.generate("c1", grid=grid, iters=iters)
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, iters, track_every=iters)
    say("fp64 volumetric", grid, "rank", ref["rank"])
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        z = run(mp, prob, "fp64", "fused", iters, ref, keep_aux=True, check_every=iters)
        f, d = mp.aux()
    assert relerr(z, ref["z"]) <= TOL["fp64"], relerr(z, ref["z"])
    assert relerr(f, ref["f"]) <= 10 * TOL["fp64"], relerr(f, ref["f"])
    assert relerr(d, ref["d"]) <= 10 * TOL["fp64"], relerr(d, ref["d"])
    assert z.min() >= 0.0


# ------------------------------------------------------------ edge cases
EDGES = [
    ("zero iters", dict(P=6, Q=5, grid=(3, 2, 1), iters=0)),
    ("single voxel", dict(P=6, Q=5, grid=(1, 1, 1), iters=25)),
    ("Q = 1", dict(P=4, Q=1, grid=(5, 3, 1), iters=25)),
    ("P > Q", dict(P=20, Q=7, grid=(4, 3, 2), iters=25)),
    ("1-D grid", dict(P=8, Q=19, grid=(37, 1, 1), iters=25)),
    ("column grid", dict(P=8, Q=33, grid=(1, 1, 23), iters=25)),
    ("ragged 3-D", dict(P=9, Q=17, grid=(13, 7, 5), iters=25)),
    ("one iteration", dict(P=9, Q=17, grid=(6, 5, 2), iters=1)),
    ("two iterations", dict(P=9, Q=17, grid=(6, 5, 2), iters=2)),
    ("rank 33 of 40", dict(P=40, Q=48, grid=(5, 4, 2), iters=20, rank=33)),
    ("P = 1", dict(P=1, Q=9, grid=(6, 4, 1), iters=25)),
    ("rank 1", dict(P=8, Q=12, grid=(5, 4, 2), iters=25, rank=1)),
]


@pytest.mark.parametrize("kernel", ["unfused", "fused", "gemm"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("label,case", EDGES, ids=[e[0] for e in EDGES])
def test_edge_cases(torch_cuda, kernel, prec, label, case):
    if kernel == "gemm" and prec == "fp64":
        pytest.skip("the GEMM path runs float32 and bf16x3")
    prob = synth.random_problem(case["P"], case["Q"], case["grid"], seed=zlib.crc32(label.encode()) % 1000,
                                lam=0.3, beta=0.5, positive_K=True)
    rank = case.get("rank", -1)
    ref = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, case["iters"], rank=rank)
    say("edge", label, prec, kernel)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        z = run(mp, prob, prec, kernel, case["iters"], ref, keep_aux=True)
        f, d = mp.aux()
    tol = TOL[prec]
    if case["iters"] == 0:
        assert not z.any() and not f.any() and not d.any()
        return
    scale = prob.beta * np.linalg.norm(ref["z"])     # d is measured against beta * ||z||
    assert relerr(z, ref["z"]) <= tol
    assert relerr(f, ref["f"]) <= 10 * tol
    assert relerr(d, ref["d"], floor=scale) <= 10 * tol


# ------------------------------------------------------------ device entry point
def test_device_solve_matches_host_and_is_deterministic(torch_cuda):
    torch = torch_cuda
    prob = synth.generate("c2", grid=(16, 12, 4), iters=30)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        zh = mp.solve(prob.m, prob.lam, prob.beta, 30, precision="fp32")
        M = torch.tensor(prob.m, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            F1 = mp.solve_torch(M, prob.lam, prob.beta, 30, precision="fp32", stream=s)
            F2 = mp.solve_torch(M, prob.lam, prob.beta, 30, precision="fp32", stream=s)
        s.synchronize()
    assert torch.equal(F1, F2)
    assert np.array_equal(F1.cpu().numpy().astype(np.float64), zh)


# ------------------------------------------------------------ failure handling
def test_errors_leave_context_usable(torch_cuda, monkeypatch):
    prob = synth.random_problem(6, 5, (3, 2, 1), seed=3)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        bad = prob.m.copy()
        bad[2, 1] = np.nan
        with pytest.raises(_ffi.SsmapError) as e:
            mp.solve(bad, 0.1, 1.0, 5)
        assert e.value.status == _ffi.SSMAP_ENONFINITE
        for kw in (dict(beta=0.0), dict(beta=-1.0)):
            with pytest.raises(_ffi.SsmapError) as e:
                mp.solve(prob.m, 0.1, kw["beta"], 5)
            assert e.value.status == _ffi.SSMAP_EINVAL
        with pytest.raises(_ffi.SsmapError) as e:
            mp.solve(prob.m, -0.1, 1.0, 5)
        assert e.value.status == _ffi.SSMAP_EINVAL
        with pytest.raises(_ffi.SsmapError) as e:
            mp.solve(prob.m, 0.1, 1.0, 5, rank=6)
        assert e.value.status == _ffi.SSMAP_EINVAL
        with pytest.raises(_ffi.SsmapError) as e:
            mp.solve(prob.m, 0.1, 1.0, -1)
        assert e.value.status == _ffi.SSMAP_EINVAL
        z = mp.solve(prob.m, 0.1, 1.0, 5)
        assert np.isfinite(z).all()
    # a budget below what the solve needs gives ENOMEM, before any allocation
    monkeypatch.setenv("SSMAP_HBM_BUDGET", "1000")
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        with pytest.raises(_ffi.SsmapError) as e:
            mp.solve(prob.m, 0.1, 1.0, 5)
        assert e.value.status == _ffi.SSMAP_ENOMEM
    monkeypatch.delenv("SSMAP_HBM_BUDGET")


def test_monitor_flags_divergence(torch_cuda):
    """A float32 overflow of the iterate is reported as ENONFINITE by the
    monitoring reduction (forced from the host with huge data)."""
    prob = synth.random_problem(6, 5, (4, 3, 1), seed=4)
    with _ffi.Mapper(prob.K, prob.grid) as mp:
        with pytest.raises(_ffi.SsmapError) as e:
            mp.solve(prob.m * 1e38, 0.1, 1e-30, 4, precision="fp32", check_every=1)
        assert e.value.status == _ffi.SSMAP_ENONFINITE
        z = mp.solve(prob.m, 0.1, 1.0, 4, precision="fp32")
        assert np.isfinite(z).all()
