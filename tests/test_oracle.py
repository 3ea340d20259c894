"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test reaches the oracle's quantity by an independent route (see
tests/pins.py), so that a plausible slip in the oracle (a dropped term, a
wrong sign, a wrong index, a transposed operand, a factor of 2) fails at
least one of them. No GPU is needed.
"""
import json
import os

import numpy as np
import pytest
import scipy.optimize

import oracle
from oracle import algorithm2 as L
import pins
from paper_2401_12890_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ------------------------------------------------------------ printed constants
def test_printed_constants_match_paper():
    """Sec. III-F constants (epsilon, 0.75, 0.005 %) as the oracle uses them."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        c = json.load(fh)
    assert L.EPS_XI == c["xi_epsilon"]["value"]
    assert L.XI_FACTOR == c["xi_factor"]["value"]
    assert L.RANK_TOL == pytest.approx(c["rank_tolerance_percent"]["value"] / 100.0, rel=0, abs=1e-18)
    # lambda = 0 leaves only epsilon in xi_p (Eq. sigma_cond)
    assert oracle.xi_rule(0.0, (5, 4, 1)) == c["xi_epsilon"]["value"]


# ------------------------------------------------------------ P2: the stencil
@pytest.mark.parametrize("grid", [(1, 1, 1), (5, 1, 1), (4, 3, 1), (3, 4, 2), (2, 3, 4)])
def test_dtd_matches_explicit_edge_list(grid):
    """D^T D z from the explicit ordered-pair D (Eq. l2) equals the oracle's."""
    N = grid[0] * grid[1] * grid[2]
    z = _rng(1).standard_normal((N, 3))
    D = pins.explicit_D(grid)
    ref = (D.T @ (D @ z))
    got = oracle.dtd_apply(z, grid)
    assert np.allclose(got, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("grid", [(4, 3, 1), (3, 2, 3)])
def test_regulariser_value_matches_double_sum(grid):
    """1/2 <z, D^T D z> equals the double sum of Eq. (l2), done with loops."""
    N = grid[0] * grid[1] * grid[2]
    z = _rng(2).standard_normal((N, 4))
    assert oracle.reg_value(z, grid) == pytest.approx(pins.R_loops(z, grid), rel=1e-13)


def test_dtd_dct_eigenvectors():
    """Separable DCT-II vectors are eigenvectors of D^T D with eigenvalue
    2 * sum_a (2 - 2 cos(pi k_a / n_a)) (free boundary on every axis)."""
    grid = (6, 5, 3)
    nx, ny, nz = grid
    for (kx, ky, kz) in [(0, 0, 0), (1, 0, 0), (5, 4, 2), (2, 3, 1)]:
        cx = np.cos(np.pi * kx * (np.arange(nx) + 0.5) / nx)
        cy = np.cos(np.pi * ky * (np.arange(ny) + 0.5) / ny)
        cz = np.cos(np.pi * kz * (np.arange(nz) + 0.5) / nz)
        v = (cz[:, None, None] * cy[None, :, None] * cx[None, None, :]).reshape(-1, 1)
        mu = 2.0 * sum(2.0 - 2.0 * np.cos(np.pi * k / n) for k, n in ((kx, nx), (ky, ny), (kz, nz)))
        assert np.allclose(oracle.dtd_apply(v, grid), mu * v, atol=1e-12)


# ------------------------------------------------------------ P3: xi_p
@pytest.mark.parametrize("grid", [(5, 4, 1), (6, 3, 2), (7, 1, 1), (1, 1, 1), (9, 8, 1)])
def test_dtd_norm_dense_vs_closed_form(grid):
    """Dense eigvalsh of the explicit D^T D equals 2 sum_a (2 + 2 cos(pi/n_a))."""
    D = pins.explicit_D(grid)
    A = (D.T @ D).toarray()
    dense = np.linalg.eigvalsh(A)[-1] if A.shape[0] > 0 else 0.0
    closed = 2.0 * sum(2.0 + 2.0 * np.cos(np.pi / n) for n in grid if n > 1)
    assert dense == pytest.approx(closed, rel=1e-12, abs=1e-12)
    assert oracle.dtd_norm(grid) == pytest.approx(closed, rel=1e-12, abs=1e-12)
    assert oracle.dtd_norm(grid, dense_limit=0) == pytest.approx(closed, rel=1e-14, abs=1e-14)


def test_xi_rule_config_values():
    """xi_p of Eq. (sigma_cond) on the three workload grids at lambda = 1e-2."""
    for grid, val in (((32, 32, 1), 0.119711), ((128, 128, 64), 0.179946),
                      ((96, 96, 32), 0.179823)):
        closed = 0.75 * 1e-2 * 2.0 * sum(2.0 + 2.0 * np.cos(np.pi / n) for n in grid if n > 1) + 1e-10
        assert oracle.xi_rule(1e-2, grid) == pytest.approx(closed, rel=1e-13)
        assert closed == pytest.approx(val, abs=5e-7)


# ------------------------------------------------------------ rank rule
def test_rank_rule_known_tails():
    s = np.array([10.0, 1.0, 1e-2, 1e-4, 1e-6])
    total = np.sqrt(np.sum(s ** 2))
    # brute force over candidate ranks with the literal definition
    want = next(r for r in range(1, 6) if np.sqrt(np.sum(s[r:] ** 2)) < 5e-5 * total)
    assert oracle.rank_rule(s, 0) == want == 3
    assert oracle.rank_rule(s, -1) == 5
    assert oracle.rank_rule(s, 2) == 2
    with pytest.raises(ValueError):
        oracle.rank_rule(s, 6)
    # strictness: a tail exactly at the threshold is not enough
    s2 = np.array([1.0, 5e-5])
    s2[0] = np.sqrt(1.0 - 5e-5 ** 2)          # ||s2|| = 1, tail = 5e-5 exactly-ish
    r = oracle.rank_rule(s2, 0)
    assert r in (1, 2)
    tail = np.sqrt(np.sum(s2[r:] ** 2))
    assert tail < 5e-5 * np.sqrt(np.sum(s2 ** 2))


def test_rank_rule_frobenius_error_of_K():
    """The chosen rank's ||K - K_r||_F is below 0.005 % and r-1 is not."""
    prob = synth.generate("c1")
    U, s, V = oracle.thin_svd(prob.K)
    r = oracle.rank_rule(s, 0)
    for rr, ok in ((r, True), (r - 1, False)):
        Kr = (U[:, :rr] * s[:rr]) @ V[:, :rr].T
        err = np.linalg.norm(prob.K - Kr) / np.linalg.norm(prob.K)
        assert (err < 5e-5) == ok


def test_thin_svd_reconstructs():
    K = _rng(3).standard_normal((7, 11))
    U, s, V = oracle.thin_svd(K)
    assert np.allclose((U * s) @ V.T, K, atol=1e-13)
    assert np.allclose(V.T @ V, np.eye(7), atol=1e-13)
    assert np.all(np.diff(s) <= 0)


# ------------------------------------------------------------ P1: the f-step
@pytest.mark.parametrize("P,Q,beta", [(12, 8, 0.5), (6, 10, 0.1), (9, 9, 2.0)])
def test_fstep_full_rank_is_exact_inverse(P, Q, beta):
    """With r = min(P, Q), Eq. (DictVecSVD) applies M = (K^T K + beta I)^{-1}
    exactly (Eq. DictMatxInv); check against a dense solve and Woodbury."""
    rng = _rng(4)
    K = rng.standard_normal((P, Q))
    c = rng.standard_normal((5, Q))
    U, s, V = oracle.thin_svd(K)
    sw = s * s / (beta * beta + beta * s * s)
    got = oracle.f_step(c, V, sw, beta)
    ref = np.linalg.solve(K.T @ K + beta * np.eye(Q), c.T).T
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    wood = (c - (K.T @ np.linalg.solve(K @ K.T + beta * np.eye(P), K @ c.T)).T) / beta
    assert np.allclose(got, wood, rtol=1e-11, atol=1e-12)


def test_fstep_solves_f_subproblem():
    """The f-update (Eqs. f2, DictMatxInv with K_r) zeroes the gradient of
    1/2||m - K_r f||^2 - <z - f, d> + beta/2 ||z - f||^2 at every voxel."""
    rng = _rng(5)
    P, Q, N, beta = 10, 14, 6, 0.3
    K = rng.standard_normal((P, Q))
    m = rng.standard_normal((N, P))
    z = np.abs(rng.standard_normal((N, Q)))
    d = rng.standard_normal((N, Q))
    U, s, V = oracle.thin_svd(K)
    r = 7
    Ur, sr, Vr = U[:, :r], s[:r], V[:, :r]
    Kr = (Ur * sr) @ Vr.T
    g = ((m @ Ur) * sr) @ Vr.T
    sw = sr * sr / (beta * beta + beta * sr * sr)
    f = oracle.f_step(g + beta * z - d, Vr, sw, beta)
    grad = (f @ Kr.T - m) @ Kr + d - beta * (z - f)
    assert np.max(np.abs(grad)) < 1e-11


# ------------------------------------------------------------ the z-step
def test_zstep_solves_z_subproblem():
    """Eq. (z2) plus clamping minimises the z-subproblem of Eq. (z) with
    P = xi I - lambda D^T D: check the projected-gradient optimality
    condition elementwise with the explicit D."""
    rng = _rng(6)
    grid = (4, 3, 2)
    N, Q = 24, 5
    lam, beta = 0.7, 0.4
    xi = 0.75 * lam * oracle.dtd_norm(grid) + 1e-10
    zk = np.abs(rng.standard_normal((N, Q)))
    f = rng.standard_normal((N, Q))
    d = rng.standard_normal((N, Q))
    z = oracle.z_step(zk, f, d, lam, xi, beta, grid)
    D = pins.explicit_D(grid)
    DtD = (D.T @ D).toarray()
    Pm = xi * np.eye(N) - lam * DtD
    # gradient of lam/2||Dz||^2 - <z - f, d> + beta/2||z - f||^2 + 1/2 (z-zk)^T P (z-zk)
    grad = lam * DtD @ z - d + beta * (z - f) + Pm @ (z - zk)
    assert np.all(z >= 0)
    pos = z > 0
    assert np.max(np.abs(grad[pos])) < 1e-12
    assert np.all(grad[~pos] >= -1e-12)


# ------------------------------------------------------------ P4: lambda = 0
def test_lambda_zero_matches_bruteforce_nnls():
    """lambda = 0 decouples Eq. (spat) into voxel-by-voxel NNLS
    (Eq. voxelbyvoxel); LADMM must reach the enumerated minimiser and the
    Lawson-Hanson answer."""
    rng = _rng(7)
    P, Q, grid = 12, 6, (3, 2, 1)
    N = 6
    K = rng.standard_normal((P, Q))
    f_true = np.maximum(0.0, rng.standard_normal((N, Q)))
    m = f_true @ K.T + 0.3 * rng.standard_normal((N, P))
    out = oracle.ladmm(K, m, grid, lam=0.0, beta=1.0, iters=3000, rank=-1)
    for n in range(N):
        bf = pins.nnls_bruteforce(K, m[n])
        lh, _ = scipy.optimize.nnls(K, m[n])
        assert np.allclose(bf, lh, atol=1e-9)
        assert np.allclose(out["z"][n], bf, atol=1e-8)
    assert np.any(out["z"] == 0.0)            # the constraint is active somewhere


# ------------------------------------------------------------ P5: interior
def test_interior_closed_form():
    """When the unconstrained minimiser of Eq. (spat) is strictly positive it
    is the constrained optimum; the LADMM limit must reach it (Q <= P, full
    column rank, so the minimiser is unique)."""
    rng = _rng(8)
    P, Q, grid = 10, 4, (3, 3, 1)
    N = 9
    K = np.abs(rng.standard_normal((P, Q))) + 0.2
    f_true = 1.0 + 0.2 * rng.uniform(size=(N, Q))
    m = f_true @ K.T
    lam = 0.05
    f_int = pins.interior_solution(K, m, grid, lam)
    assert f_int.min() > 0.1
    out = oracle.ladmm(K, m, grid, lam=lam, beta=2.0, iters=4000, rank=-1)
    assert np.allclose(out["z"], f_int, atol=1e-9)
    assert np.allclose(out["f"], f_int, atol=1e-9)


# ------------------------------------------------------------ P6/P7: KKT + FISTA
@pytest.fixture(scope="module")
def converged_small():
    rng = _rng(9)
    P, Q, grid = 8, 6, (3, 3, 1)
    N = 9
    K = rng.standard_normal((P, Q))
    f_true = np.maximum(0.0, rng.standard_normal((N, Q)))
    m = f_true @ K.T + 0.2 * rng.standard_normal((N, P))
    lam = 0.3
    out = oracle.ladmm(K, m, grid, lam=lam, beta=1.0, iters=6000, rank=-1)
    return K, m, grid, lam, out


def test_kkt_at_convergence(converged_small):
    K, m, grid, lam, out = converged_small
    zmin, compl, _ = pins.kkt_residual(K, m, out["z"], grid, lam)
    assert zmin >= 0.0
    assert compl < 1e-8
    assert np.max(np.abs(out["z"] - out["f"])) < 1e-8
    assert np.any(out["z"] == 0.0)


def test_objective_matches_projected_gradient(converged_small):
    K, m, grid, lam, out = converged_small
    x, Jf = pins.fista(K, m, grid, lam)
    J_ladmm = oracle.objective(K, m, out["z"], grid, lam)
    assert J_ladmm == pytest.approx(Jf, rel=1e-8)
    assert J_ladmm == pytest.approx(pins.J_explicit(K, m, out["z"], grid, lam), rel=1e-12)
    assert np.allclose(out["z"], x, atol=1e-6)


# ------------------------------------------------------------ P8: fixed point
def test_fixed_point_is_kkt_point(converged_small):
    """Seed (z*, d* = K^T (m - K z*)) from the independent solver: one LADMM
    step must leave it unchanged (the whole iteration is pinned at once)."""
    K, m, grid, lam, _ = converged_small
    x, _ = pins.fista(K, m, grid, lam)
    d_star = (m - x @ K.T) @ K
    out = oracle.ladmm(K, m, grid, lam=lam, beta=0.7, iters=1, rank=-1, z0=x, d0=d_star)
    assert np.allclose(out["z"], x, atol=1e-9)
    assert np.allclose(out["d"], d_star, atol=1e-9)
    assert np.allclose(out["f"], x, atol=1e-9)


# ------------------------------------------------------------ P9: invariants
def test_invariants():
    prob = synth.random_problem(9, 7, (4, 3, 2), seed=10, lam=0.2, beta=0.5)
    base = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, 20, rank=5)
    # positive homogeneity in m
    sc = oracle.ladmm(prob.K, 3.0 * prob.m, prob.grid, prob.lam, prob.beta, 20, rank=5)
    assert np.allclose(sc["z"], 3.0 * base["z"], rtol=1e-12, atol=1e-12)
    # spatial flip along x
    nx, ny, nz = prob.grid
    Q = prob.Q
    m4 = prob.m.reshape(nz, ny, nx, -1)[:, :, ::-1, :].reshape(prob.N, -1)
    fl = oracle.ladmm(prob.K, m4, prob.grid, prob.lam, prob.beta, 20, rank=5)
    z4 = base["z"].reshape(nz, ny, nx, Q)[:, :, ::-1, :].reshape(prob.N, Q)
    assert np.allclose(fl["z"], z4, atol=1e-12)
    # permutation of the dictionary columns permutes the output
    perm = _rng(11).permutation(Q)
    pm = oracle.ladmm(prob.K[:, perm], prob.m, prob.grid, prob.lam, prob.beta, 20, rank=5)
    assert np.allclose(pm["z"], base["z"][:, perm], atol=1e-11)


# ------------------------------------------------------------ P10: degenerate
def test_degenerate_cases():
    rng = _rng(12)
    # iters = 0 -> zeros
    K = rng.standard_normal((5, 4))
    m = rng.standard_normal((6, 5))
    out = oracle.ladmm(K, m, (3, 2, 1), 0.1, 1.0, 0)
    assert not out["z"].any()
    # N = 1: D = 0, the problem is a single NNLS
    m1 = m[:1]
    o1 = oracle.ladmm(K, m1, (1, 1, 1), 5.0, 1.0, 3000, rank=-1)
    lh, _ = scipy.optimize.nnls(K, m1[0])
    assert np.allclose(o1["z"][0], lh, atol=1e-8)
    # Q = 1: scalar Tikhonov-NNLS, compare with the dense interior/boundary solve
    k = np.abs(rng.standard_normal((4, 1))) + 0.5
    grid = (3, 1, 1)
    mq = np.array([[1.0], [2.0], [-3.0]]) @ k.T
    oq = oracle.ladmm(k, mq, grid, 0.1, 1.0, 5000, rank=-1)
    x, _ = pins.fista(k, mq, grid, 0.1)
    assert np.allclose(oq["z"], x, atol=1e-8)


def test_dfcs_history_monotone_objective():
    prob = synth.generate("c1", grid=(8, 8, 1))
    out = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, 60, track_every=10)
    J = [h[1] for h in out["hist"]]
    assert J[-1] < J[0]
    assert len(out["hist"]) == 7


@pytest.mark.parametrize("workload,nsamples", [("c2", 2), ("c3x", 1)])
def test_fullsize_golden_values_come_from_the_oracle(workload, nsamples):
    """The stored full-size sample values (used by the benchmark) are what the
    oracle gives on crops: recompute some of them (c3x: the c3 recipe at the
    unapproximated rank min(P, Q))."""
    import importlib.util
    path = os.path.join(GOLDEN, "make_fullsize_golden.py")
    spec = importlib.util.spec_from_file_location("make_fullsize_golden", path)
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    with open(os.path.join(GOLDEN, f"fullsize_{workload}.json")) as fh:
        gold = json.load(fh)
    recipe, rank_param = mk.WORKLOADS[workload]
    prob = synth.generate(recipe)
    assert gold["rank"] == oracle.rank_rule(oracle.thin_svd(prob.K)[1], rank_param)
    if rank_param == -1:
        assert gold["rank"] == min(prob.P, prob.Q)
    g = np.random.Generator(np.random.PCG64(gold["projection_seed"])).standard_normal(prob.Q)
    nx, ny, nz = prob.grid
    h = gold["iters"] + 1
    for smp in gold["samples"][:nsamples]:
        x, y, z = smp["voxel"]
        x0, x1 = max(0, x - h), min(nx, x + h + 1)
        y0, y1 = max(0, y - h), min(ny, y + h + 1)
        z0, z1 = max(0, z - h), min(nz, z + h + 1)
        idx = [xx + nx * (yy + ny * zz) for zz in range(z0, z1) for yy in range(y0, y1)
               for xx in range(x0, x1)]
        sub = oracle.ladmm(prob.K, prob.m[idx], (x1 - x0, y1 - y0, z1 - z0), prob.lam, prob.beta,
                           gold["iters"], rank=gold["rank"], xi=gold["xi_p"])
        zr = sub["z"][(x - x0) + (x1 - x0) * ((y - y0) + (y1 - y0) * (z - z0))]
        assert np.linalg.norm(zr) == pytest.approx(smp["norm"], rel=1e-12)
        assert zr @ g == pytest.approx(smp["proj"], rel=1e-10, abs=1e-14)
    assert [s["voxel"] for s in gold["samples"]] == [list(p) for p in mk.points(prob.grid)]


def test_iters300_golden_files_are_consistent_with_their_script_and_rules():
    """The stored oracle results at the configured iteration counts carry the rank
    of the oracle's rule on the recipe's dictionary (it does not depend on the
    grid), the xi_p rule's value on the full grid, the recipe's lambda and beta
    and the script's sample voxels; their sums agree with each other and with the
    sampled Q-vectors (a mix-up of stored arrays fails here). The 300-iteration
    3-D files are too long to recompute here; the 32 x 32 file (500 iterations,
    about a second) is recomputed and must match."""
    import importlib.util
    path = os.path.join(GOLDEN, "make_iters300_golden.py")
    spec = importlib.util.spec_from_file_location("make_iters300_golden", path)
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    for case, cfg in mk.CASES.items():
        g = np.load(os.path.join(GOLDEN, mk.file_name(case)))
        grid = tuple(int(v) for v in g["grid"])
        small = synth.generate(cfg["recipe"], grid=(4, 4, 2))
        if cfg["grid"] is not None:
            assert grid == tuple(cfg["grid"])
        assert int(g["iters"]) == cfg["iters"]
        assert int(g["rank"]) == oracle.rank_rule(oracle.thin_svd(small.K)[1], 0)
        assert float(g["xi_p"]) == oracle.xi_rule(small.lam, grid)
        assert float(g["lam"]) == small.lam and float(g["beta"]) == small.beta
        pts = mk.sample_voxels(grid, cfg["brick"])
        nx, ny, _ = grid
        assert np.array_equal(g["index"], [x + nx * (y + ny * z) for (x, y, z) in pts])
        total = float(g["z_sum_q"].sum())
        assert float(g["z_sum_n"].sum()) == pytest.approx(total, rel=1e-12)
        assert float(np.sqrt((g["z_norm_q"] ** 2).sum())) == pytest.approx(float(g["norm_z"]), rel=1e-12)
        np.testing.assert_allclose(g["z"].sum(axis=1), g["z_sum_q"][g["index"]], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(np.linalg.norm(g["z"], axis=1), g["z_norm_q"][g["index"]],
                                   rtol=1e-12, atol=1e-15)
        if case == "c1":
            prob = synth.generate("c1")
            out = oracle.ladmm(prob.K, prob.m, prob.grid, prob.lam, prob.beta, cfg["iters"])
            np.testing.assert_allclose(out["z"][g["index"]], g["z"], rtol=0, atol=1e-13)
            np.testing.assert_allclose(out["z"].sum(axis=1), g["z_sum_q"], rtol=1e-13, atol=1e-15)
            assert float(np.linalg.norm(out["z"])) == pytest.approx(float(g["norm_z"]), rel=1e-13)


def test_batch200_golden_values_come_from_the_oracle():
    """The stored configured-batch values are the oracle's: recompute the smallest
    stored slice (4,320 voxels, Q = 100) at the configured 200 iterations, and
    check the other stored slices' sample indices and ranks against the generator
    and the rank rule."""
    import importlib.util
    path = os.path.join(GOLDEN, "make_batch200_golden.py")
    spec = importlib.util.spec_from_file_location("make_batch200_golden", path)
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    g = np.load(os.path.join(GOLDEN, "batch200_c4.npz"))
    probs = synth.generate_batch()
    chosen = mk.chosen_slices(probs)
    assert [p.meta["slice"] for p in chosen] == [int(k) for k in g["slices"]]
    for p in chosen:
        k = p.meta["slice"]
        assert np.array_equal(g[f"s{k}_index"], mk.sample_voxels(p.grid))
        assert int(g[f"s{k}_rank"]) == oracle.rank_rule(oracle.thin_svd(p.K)[1], 0)
    p = min(chosen, key=lambda p: p.N)
    k = p.meta["slice"]
    ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, int(g["iters"]))
    np.testing.assert_allclose(ref["z"][g[f"s{k}_index"]], g[f"s{k}_z"], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(ref["z"].sum(axis=1), g[f"s{k}_z_sum_q"], rtol=1e-10, atol=1e-13)
    assert float(np.linalg.norm(ref["z"])) == pytest.approx(float(g[f"s{k}_norm_z"]), rel=1e-12)


def test_bench_uses_the_oracle_only_in_its_cpu_baseline():
    import ast
    src = open(os.path.join(os.path.dirname(GOLDEN), "..", "bench.py")).read()
    tree = ast.parse(src)
    users = set()
    for fn in [n for n in ast.walk(tree) if isinstance(n, ast.FunctionDef)]:
        for node in ast.walk(fn):
            if isinstance(node, (ast.Import, ast.ImportFrom)):
                names = [a.name for a in node.names] + [getattr(node, "module", None) or ""]
                if any(nm.split(".")[0] == "oracle" for nm in names):
                    users.add(fn.name)
    assert users and all(u.startswith("cpu_baseline") for u in users)
