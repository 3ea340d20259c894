"""Masked voxel sets, the residual stopping rule and the penalty heuristic on
the GPU, through the C ABI, against the FP64 oracle.

Masks: only inside voxels are estimated (Sec. II-C, maskless footnote); the
oracle solves the same problem on the graph of inside face neighbours.
"""
import numpy as np
import pytest

import oracle
from paper_2401_12890_amd import _ffi, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-3}


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
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def ellipsoid_mask(grid, centre, radii, holes=0, seed=0):
    """An ellipsoid of inside voxels, optionally with single-voxel holes."""
    nx, ny, nz = grid
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = sum(((c - c0) / max(rr, 1e-9)) ** 2 for c, c0, rr in zip((x, y, z), centre, radii))
    m = (r2 <= 1.0).reshape(-1)
    if holes:
        rng = np.random.Generator(np.random.PCG64(seed))
        idx = np.flatnonzero(m)
        m[rng.choice(idx, size=min(holes, idx.size // 4), replace=False)] = False
    return m


CASES = [
    # name, recipe, grid, centre, radii, holes, iters
    ("planar disk", "c1", (37, 29, 1), (18, 14, 0), (15, 11, 1), 6, 40),
    ("3-D ellipsoid", "c2", (21, 19, 9), (10, 9, 4), (9, 8, 5), 8, 25),
    ("small blob in a large box", "c3", (70, 40, 6), (12, 10, 2), (6, 5, 3), 0, 20),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("name,recipe,grid,centre,radii,holes,iters", CASES,
                         ids=[c[0] for c in CASES])
def test_masked_solve_matches_oracle(torch_cuda, name, recipe, grid, centre, radii, holes, iters,
                                     prec):
    p = synth.generate(recipe, grid=grid, iters=iters)
    mask = ellipsoid_mask(grid, centre, radii, holes)
    m = p.m.copy()
    m[~mask] = np.nan                                 # outside rows are never read
    ref = oracle.ladmm(p.K, m, p.grid, p.lam, p.beta, iters, mask=mask)
    say(name, prec, "inside", int(mask.sum()), "of", p.N, "rank", ref["rank"])
    with _ffi.Mapper(p.K, p.grid) as mp:
        mp.set_mask(mask)
        for kernel in ("unfused", "fused"):
            F = mp.solve(m, p.lam, p.beta, iters, precision=prec, kernel=kernel)
            st = mp.stats()
            assert abs(st["dtd_norm"] - (ref["xi"] - 1e-10) / (0.75 * p.lam)) <= 1e-9 * st["dtd_norm"]
            assert np.all(F[~mask] == 0.0)
            err = relerr(F, ref["z"])
            say("  ", kernel, err)
            assert err <= TOL[prec], (name, prec, kernel, err)


# Masked grids with short spectra on the double-buffered bricks: the brick
# table holds only bricks with an inside voxel (still more than the CUs), and
# the persistent grid walks it. Float32 volumetric 16 x 8 x 4 (Q = 36) and
# float64 planar 16 x 8 x 1 (Q = 100).
WALK_CASES = [
    ("c2", (70, 66, 40), (34, 32, 19), (33, 31, 19), "fp32", 6),
    ("c1", (300, 200, 1), (150, 100, 0), (148, 98, 1), "fp64", 10),
]


@pytest.mark.parametrize("recipe,grid,centre,radii,prec,n", WALK_CASES)
def test_masked_persistent_walk(torch_cuda, recipe, grid, centre, radii, prec, n):
    iters = 10
    p = synth.generate(recipe, grid=grid, iters=iters, overrides=dict(n1=n, n2=n))
    mask = ellipsoid_mask(grid, centre, radii, holes=40, seed=5)
    m = p.m.copy()
    m[~mask] = np.nan
    ref = oracle.ladmm(p.K, m, p.grid, p.lam, p.beta, iters, mask=mask)
    say("masked walk", recipe, grid, prec, "inside", int(mask.sum()), "of", p.N, "rank", ref["rank"])
    with _ffi.Mapper(p.K, p.grid) as mp:
        mp.set_mask(mask)
        F = mp.solve(m, p.lam, p.beta, iters, precision=prec, kernel="fused")
    assert np.all(F[~mask] == 0.0)
    err = relerr(F, ref["z"])
    assert err <= TOL[prec], (recipe, grid, prec, err)


def test_mask_norm_objective_and_reset(torch_cuda):
    p = synth.generate("c1", grid=(23, 17, 1), iters=30)
    mask = ellipsoid_mask(p.grid, (11, 8, 0), (10, 7, 1), holes=5, seed=3)
    ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 30, mask=mask)
    edges = oracle.graph_edges(p.grid, mask)
    with _ffi.Mapper(p.K, p.grid) as mp:
        mp.set_mask(mask)
        F = mp.solve(p.m, p.lam, p.beta, 30, precision="fp64", check_every=10)
        st = mp.stats()
        assert abs(st["dtd_norm"] - oracle.dtd_norm_graph(edges, int(mask.sum()))) <= 1e-10 * st["dtd_norm"]
        J = oracle.objective_masked(ref["K_r"], p.m, ref["z"], p.grid, p.lam, mask)
        assert abs(st["hist_objective"][-1] - J) <= 1e-9 * J
        assert relerr(F, ref["z"]) <= 1e-10
        # back to the whole box
        mp.set_mask(None)
        F2 = mp.solve(p.m, p.lam, p.beta, 30, precision="fp64")
        ref2 = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 30)
        assert relerr(F2, ref2["z"]) <= 1e-10
        # a mask with no inside voxel gives zeros
        mp.set_mask(np.zeros(p.N, dtype=bool))
        F3 = mp.solve(p.m, p.lam, p.beta, 5, precision="fp32")
        assert np.all(F3 == 0.0)


@pytest.mark.parametrize("prec,tol,every", [("fp64", 1e-3, 5), ("fp64", 0.25, 1), ("fp32", 2e-3, 10)])
def test_stopping_rule_matches_oracle(torch_cuda, prec, tol, every):
    p = synth.generate("c1", grid=(14, 11, 1))
    ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 400, stop_tol=tol, check_every=every)
    with _ffi.Mapper(p.K, p.grid) as mp:
        F = mp.solve(p.m, p.lam, p.beta, 400, precision=prec, check_every=every, stop_tol=tol)
        st = mp.stats()
    say(prec, tol, every, "stopped at", st["iters"], "oracle", ref["iters"])
    assert st["iters"] == ref["iters"] < 400
    assert relerr(F, ref["z"]) <= TOL[prec]


def test_stopping_rule_argument_errors(torch_cuda):
    p = synth.generate("c1", grid=(6, 5, 1))
    with _ffi.Mapper(p.K, p.grid) as mp:
        for kw in (dict(stop_tol=1e-3), dict(stop_tol=-1.0, check_every=2),
                   dict(stop_tol=1e-3, check_every=2, keep_aux=True)):
            with pytest.raises(_ffi.SsmapError) as e:
                mp.solve(p.m, p.lam, p.beta, 10, **kw)
            assert e.value.status == _ffi.SSMAP_EINVAL


@pytest.mark.parametrize("recipe,grid,prec", [("c1", (12, 10, 1), "fp64"),
                                              ("c2", (9, 8, 5), "fp32")])
def test_beta_heuristic_matches_oracle(torch_cuda, recipe, grid, prec):
    p = synth.generate(recipe, grid=grid)
    betas = [1e-3, 1e-2, 1e-1, 1.0, 10.0]
    iters = 60
    best_o, J_o = oracle.beta_heuristic(p.K, p.m, p.grid, p.lam, iters, betas)
    with _ffi.Mapper(p.K, p.grid) as mp:
        best, J = mp.tune_beta(p.m, p.lam, iters, betas, precision=prec)
    say(recipe, prec, "oracle", best_o, J_o, "gpu", best, J)
    rel = 1e-9 if prec == "fp64" else 1e-4
    assert np.all(np.abs(J - J_o) <= rel * J_o)
    order = np.argsort(J_o)
    if J_o[order[1]] - J_o[order[0]] > 10 * rel * J_o[order[0]]:
        assert best == best_o
