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


def test_admm_fixed_point_is_left_unchanged():
    """Algorithm 1 seeded at the minimiser z* (from FISTA, an independent
    solver) with f = x = y = z = z* and the duals that the x-, y- and z-steps
    imply there -- d_x = K^T (m - K z*), d_y = grad J(z*) (>= 0, zero where
    z* > 0 by the KKT conditions), d_z = -lambda D^T D z* (so the three sum to
    zero) -- stays where it is after one iteration."""
    grid = (4, 3, 2)
    K, m, lam = smooth_problem(grid, seed=13)
    beta = 0.7
    zs, _ = pins.fista(K, m, grid, lam)
    D = pins.explicit_D(grid)
    DtD = (D.T @ D).tocsr()
    dx = (m - zs @ K.T) @ K
    dz = -lam * (DtD @ zs)
    dy = pins.grad_J(K, m, zs, grid, lam)
    assert np.abs(dx + dy + dz).max() <= 1e-12 * np.abs(dx).max()
    seed = dict(f=zs, x=zs, y=zs, z=zs, dx=dx, dy=dy, dz=dz)
    out = oracle.admm_previous(K, m, grid, lam, beta, 1, init=seed)
    scale = np.linalg.norm(zs)
    for k in ("f", "x", "y", "z"):
        assert np.linalg.norm(out[k] - zs) <= 1e-8 * scale, k
    for k in ("dx", "dy", "dz"):
        assert np.linalg.norm(out[k] - seed[k]) <= 1e-8 * beta * scale, k


def test_admm_first_iterates_in_closed_form():
    """From zero, Algorithm 1's first two iterations and the third f-step
    written out by hand (dense solves with the explicit D instead of the
    oracle's inverse and DCT), which fixes the order of the updates:
      k=1: f = 0, x = M K^T m =: x1, y = z = 0, d_x = beta x1, d_y = d_z = 0;
      k=2: f = 2 x1 / 3, x = M (K^T m - beta x1 / 3), y = max(0, 2 x1 / 3),
           z = (lambda D^T D + beta I)^{-1} (2 beta x1 / 3),
           d_x = beta x1 - beta (f - x), d_y = -beta (f - y), d_z = -beta (f - z);
      k=3: f = (beta x + d_x + beta y + d_y + beta z + d_z) / (3 beta) of those."""
    grid = (3, 3, 2)
    rng = np.random.Generator(np.random.PCG64(21))
    P, Q = 9, 5
    K = rng.standard_normal((P, Q))
    N = int(np.prod(grid))
    m = rng.standard_normal((N, P))              # signed data: x1 has both signs
    lam, beta = 0.4, 0.9
    Mi = np.linalg.solve(K.T @ K + beta * np.eye(Q), np.eye(Q))
    D = pins.explicit_D(grid).toarray()
    A = lam * D.T @ D + beta * np.eye(N)
    x1 = (m @ K) @ Mi.T
    o1 = oracle.admm_previous(K, m, grid, lam, beta, 1)
    ref1 = dict(f=0 * x1, x=x1, y=0 * x1, z=0 * x1, dx=beta * x1, dy=0 * x1, dz=0 * x1)
    for k, v in ref1.items():
        assert np.allclose(o1[k], v, rtol=0, atol=1e-12), k
    f2 = 2.0 * x1 / 3.0
    x2 = (m @ K - beta * x1 / 3.0) @ Mi.T
    y2 = np.maximum(0.0, f2)
    z2 = np.linalg.solve(A, beta * f2)
    ref2 = dict(f=f2, x=x2, y=y2, z=z2, dx=beta * x1 - beta * (f2 - x2), dy=-beta * (f2 - y2),
                dz=-beta * (f2 - z2))
    assert (x1 < 0).any() and (x1 > 0).any()
    o2 = oracle.admm_previous(K, m, grid, lam, beta, 2)
    for k, v in ref2.items():
        assert np.allclose(o2[k], v, rtol=0, atol=1e-12), k
    f3 = (beta * x2 + ref2["dx"] + beta * y2 + ref2["dy"] + beta * z2 + ref2["dz"]) / (3.0 * beta)
    o3 = oracle.admm_previous(K, m, grid, lam, beta, 3)
    assert np.allclose(o3["f"], f3, rtol=0, atol=1e-12)


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


# ------------------------------------------------------------- monitored quantities
def test_primal_residual_history_equals_the_dual_step():
    """The oracle's primal residual ||z^k - f^k|| equals ||d^k - d^{k-1}|| / beta
    (the dual update of Algorithm 2 read backwards), from two fixed-length
    runs; DFCS of f^k and z^k follow Eq. (DFCS) against a reference."""
    p = synth.generate("c1", grid=(7, 5, 1))
    f_star = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 400, rank=-1)["z"]
    out = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, 30, track_every=10, f_star=f_star)
    assert [h[0] for h in out["hist_f"]] == [0, 10, 20, 30]
    for (k, primal, dfcs_f), (k2, _, dfcs_z) in zip(out["hist_f"], out["hist"]):
        assert k == k2
        if k == 0:
            assert primal == 0.0
            continue
        a = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, k - 1)
        b = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, k)
        ref = np.linalg.norm(b["d"] - a["d"]) / p.beta
        assert abs(primal - ref) <= 1e-10 * max(ref, 1e-300)
        assert dfcs_f == pytest.approx(np.linalg.norm(b["f"] - f_star) / np.linalg.norm(f_star),
                                       rel=1e-14)
        assert dfcs_z == pytest.approx(np.linalg.norm(b["z"] - f_star) / np.linalg.norm(f_star),
                                       rel=1e-14)
