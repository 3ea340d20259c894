"""Pins of the oracle's extensions: the previous ADMM (Algorithm 1), masked
voxel sets, the residual stopping rule and the penalty heuristic (Sec. III-F).

As in test_oracle.py, every check reaches the quantity by a route other than
the oracle's own code (explicit sparse D, dense solves, FISTA, slicing)."""
import numpy as np
import pytest

import oracle
from paper_2401_12890_amd import synth
from tests import pins


def smooth_problem(grid, P=12, Q=6, seed=7, lam=0.05):
    """Q <= P with full column rank: the minimiser of Eq. (spat) is unique."""
    rng = np.random.Generator(np.random.PCG64(seed))
    K = rng.uniform(0.0, 1.0, (P, Q))
    N = int(np.prod(grid))
    f = np.abs(rng.standard_normal((N, Q)))
    m = f @ K.T + 0.05 * rng.standard_normal((N, P))
    return K, m, lam


# ------------------------------------------------------------- previous ADMM
@pytest.mark.parametrize("grid", [(5, 4, 1), (4, 3, 3), (7, 1, 1)])
def test_admm_z_solve_matches_dense_solve(grid):
    rng = np.random.Generator(np.random.PCG64(3))
    N = int(np.prod(grid))
    b = rng.standard_normal((N, 3))
    lam, beta = 0.7, 0.3
    D = pins.explicit_D(grid).toarray()
    A = lam * D.T @ D + beta * np.eye(N)
    ref = np.linalg.solve(A, b)
    got = oracle.z_solve_dct(b, grid, lam, beta)
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_admm_and_ladmm_reach_the_same_minimiser():
    grid = (4, 3, 2)
    K, m, lam = smooth_problem(grid)
    zf, Jf = pins.fista(K, m, grid, lam)
    a = oracle.admm_previous(K, m, grid, lam, beta=1.0, iters=3000)
    b = oracle.ladmm(K, m, grid, lam, beta=1.0, iters=3000, rank=-1)
    for z in (a["y"], b["z"]):
        assert np.linalg.norm(z - zf) <= 1e-6 * np.linalg.norm(zf)
        assert abs(pins.J_explicit(K, m, z, grid, lam) - Jf) <= 1e-9 * Jf
    # the four copies of f in Algorithm 1 agree at convergence
    for k in ("x", "z", "f"):
        assert np.linalg.norm(a[k] - a["y"]) <= 1e-6 * np.linalg.norm(a["y"])


def test_admm_keeps_eight_image_sized_arrays():
    grid = (3, 2, 1)
    K, m, lam = smooth_problem(grid)
    out = oracle.admm_previous(K, m, grid, lam, 1.0, 2)
    N, Q = int(np.prod(grid)), K.shape[1]
    state = [v for v in out.values() if v.shape == (N, Q)]
    assert len(state) + 1 == 8                       # f, x, y, z, dx, dy, dz and g


# ------------------------------------------------------------- masked voxel sets
def blob_mask(grid, seed=5, frac=0.6):
    rng = np.random.Generator(np.random.PCG64(seed))
    inside = rng.uniform(size=int(np.prod(grid))) < frac
    inside[0] = True
    return inside


@pytest.mark.parametrize("grid", [(6, 5, 1), (4, 4, 3)])
def test_graph_stencil_matches_explicit_masked_D(grid):
    mask = blob_mask(grid)
    D = pins.explicit_D_masked(grid, mask)
    edges = oracle.graph_edges(grid, mask)
    n = int(mask.sum())
    z = np.random.Generator(np.random.PCG64(1)).standard_normal((n, 5))
    assert np.allclose(oracle.dtd_apply_graph(z, edges), (D.T @ D) @ z, atol=1e-13)
    # full mask: the graph stencil is the box stencil
    full = np.ones(int(np.prod(grid)), dtype=bool)
    zf = np.random.Generator(np.random.PCG64(2)).standard_normal((full.size, 3))
    assert np.allclose(oracle.dtd_apply_graph(zf, oracle.graph_edges(grid, full)),
                       oracle.dtd_apply(zf, grid), atol=1e-13)


@pytest.mark.parametrize("grid", [(6, 5, 1), (5, 4, 3)])
def test_graph_norm_dense_and_sparse_routes(grid):
    mask = blob_mask(grid, seed=9, frac=0.7)
    D = pins.explicit_D_masked(grid, mask).toarray()
    ref = float(np.linalg.eigvalsh(D.T @ D)[-1])
    edges = oracle.graph_edges(grid, mask)
    n = int(mask.sum())
    assert abs(oracle.dtd_norm_graph(edges, n) - ref) <= 1e-12 * ref
    assert abs(oracle.dtd_norm_graph(edges, n, dense_limit=1) - ref) <= 1e-9 * ref


def test_masked_ladmm_converges_to_masked_fista_and_ignores_outside():
    grid = (5, 4, 2)
    K, m, lam = smooth_problem(grid, seed=11)
    mask = blob_mask(grid, seed=4, frac=0.55)
    m_bad = m.copy()
    m_bad[~mask] = np.nan                            # outside data is never read
    out = oracle.ladmm(K, m_bad, grid, lam, 1.0, 4000, rank=-1, mask=mask)
    D = pins.explicit_D_masked(grid, mask)
    zf, Jf = pins.fista(K, m[mask], grid, lam, D=D)
    assert np.all(out["z"][~mask] == 0.0)
    assert np.linalg.norm(out["z"][mask] - zf) <= 1e-6 * np.linalg.norm(zf)
    J = oracle.objective_masked(out["K_r"], m, out["z"], grid, lam, mask)
    assert abs(J - Jf) <= 1e-9 * Jf


def test_full_mask_equals_the_box():
    p = synth.generate("c1", grid=(7, 6, 1), iters=25)
    full = np.ones(p.N, dtype=bool)
    a = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 25)
    b = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 25, mask=full)
    assert abs(a["xi"] - b["xi"]) <= 1e-12 * a["xi"]
    assert np.linalg.norm(a["z"] - b["z"]) <= 1e-12 * np.linalg.norm(a["z"])


# ------------------------------------------------------------- stopping rule
@pytest.mark.parametrize("tol,every", [(1e-3, 5), (0.25, 1)])
def test_stopping_rule_stops_at_the_first_passing_check(tol, every):
    p = synth.generate("c1", grid=(6, 5, 1))
    out = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 400, stop_tol=tol, check_every=every)
    k = out["iters"]
    assert k % every == 0 and k < 400
    # recompute the relative changes at every check by plain fixed-length runs
    def change(n):
        z1 = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, n - 1)["z"]
        z2 = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, n)["z"]
        return np.linalg.norm(z2 - z1) / np.linalg.norm(z2), z2
    c, z = change(k)
    assert c <= tol and np.array_equal(z, out["z"])
    if k > every:
        assert change(k - every)[0] > tol


# ------------------------------------------------------------- penalty heuristic
def test_centre_patch_and_patch_data_by_slicing():
    grid = (9, 7, 4)
    origin, pgrid = oracle.centre_patch(grid)
    assert origin == (3, 2, 0) and pgrid == (3, 3, 3)
    assert oracle.centre_patch((2, 10, 1)) == ((0, 3, 0), (2, 3, 1))
    m = np.arange(np.prod(grid) * 2, dtype=np.float64).reshape(-1, 2)
    cube = m.reshape(grid[2], grid[1], grid[0], 2)
    ref = cube[origin[2]:origin[2] + 3, origin[1]:origin[1] + 3, origin[0]:origin[0] + 3]
    assert np.array_equal(oracle.patch_data(m, grid, origin, pgrid), ref.reshape(-1, 2))


def test_beta_heuristic_picks_the_lowest_patch_objective():
    p = synth.generate("c1", grid=(12, 10, 1))
    betas = [1e-3, 1e-2, 1e-1, 1.0, 10.0]
    best, J = oracle.beta_heuristic(p.K, p.m, p.grid, p.lam, 60, betas)
    origin, pgrid = oracle.centre_patch(p.grid)
    mp = oracle.patch_data(p.m, p.grid, origin, pgrid)
    for b, Jb in zip(betas, J):
        out = oracle.ladmm(p.K, mp, pgrid, p.lam, b, 60)
        assert abs(pins.J_explicit(out["K_r"], mp, out["z"], pgrid, p.lam) - Jb) <= 1e-10 * Jb
    assert best == betas[int(np.argmin(J))]
    # a converged patch objective bounds every candidate from below
    zf, Jf = pins.fista(oracle.ladmm(p.K, mp, pgrid, p.lam, 1.0, 1)["K_r"], mp, pgrid, p.lam)
    assert np.all(J >= Jf * (1 - 1e-9))
