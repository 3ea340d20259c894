"""FP64 CPU oracle: Algorithm 2 (LADMM) of the paper, step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring). Everything here is
float64 NumPy; library primitives (SVD, matrix products, eigvalsh) serve as
single steps, with no blocking, fusion or reordering beyond what the paper's
definitions state.

Array conventions: a spectroscopic image f (and z, d, g, c) is stored
voxel-major as an (N, Q) array whose row n is f_n; data m is (N, P); the box
grid is (nx, ny, nz) with voxel n = x + nx*(y + ny*z).

Readings of points the paper leaves open (each is also listed in the design
notes of the repository):
  * Regulariser (Eq. l2, Sec. II-C): R(f) sums 1/2 ||f_n - f_m||^2 over every
    voxel n and every face neighbour m of n, so each adjacent pair appears
    twice and D has one row per ordered pair. Hence D^T D = 2 L with L the
    graph Laplacian of the grid, and (D^T D z)_n = 2 sum_m (z_n - z_m).
  * Neighbourhood: face neighbours (4 in 2-D, 6 in 3-D), unit weight per axis,
    free (Neumann) boundary: edge voxels simply have fewer neighbours.
  * The map returned after a fixed number of iterations is z^K (the feasible
    iterate); f^K and d^K are returned too.
  * g uses the rank-r factors as Algorithm 2 does, so the iteration minimises
    the problem with K replaced by K_r; the objective here takes K_r likewise.
  * Rank rule (Sec. III-F): smallest r whose relative Frobenius error
    ||K - K_r||_F / ||K||_F is strictly below 0.005 % (5e-5).
  * xi_p (Eq. sigma_cond): 0.75 * lambda * ||D^T D||_2 + 1e-10, spectral norm.
"""
from __future__ import annotations

import numpy as np

EPS_XI = 1e-10          # epsilon of Eq. (sigma_cond)
XI_FACTOR = 0.75        # 0.75 factor of the convergence condition (Sec. III-F)
RANK_TOL = 5e-5         # 0.005 % Frobenius approximation error (Sec. III-F)


# --------------------------------------------------------------- dictionary
def thin_svd(K: np.ndarray):
    """Thin SVD K = U diag(s) V^T via LAPACK (Algorithm 2, SVD step).

    Returns U (P, k), s (k,), V (Q, k) with k = min(P, Q), s descending."""
    U, s, Vt = np.linalg.svd(np.asarray(K, dtype=np.float64), full_matrices=False)
    return U, s, Vt.T


def rank_rule(s: np.ndarray, rank: int = 0) -> int:
    """Rank r (Sec. III-F, rank parameter).

    rank > 0: that rank; rank == -1: min(P, Q) (the unapproximated K);
    rank == 0: smallest r with ||K - K_r||_F < 5e-5 ||K||_F."""
    k = len(s)
    if rank == -1:
        return k
    if rank > 0:
        if rank > k:
            raise ValueError("rank exceeds min(P, Q)")
        return rank
    total = float(np.sum(s * s))
    for r in range(1, k + 1):
        tail = float(np.sum(s[r:] * s[r:]))
        if np.sqrt(tail) < RANK_TOL * np.sqrt(total):
            return r
    return k


# --------------------------------------------------------------- regulariser
def dtd_apply(z: np.ndarray, grid) -> np.ndarray:
    """D^T D z for the finite-difference operator of Eq. (l2).

    Per axis, every adjacent pair (i, i+1) adds (z_i - z_{i+1}) to voxel i and
    (z_{i+1} - z_i) to voxel i+1; the factor 2 comes from each pair being
    counted from both of its voxels."""
    nx, ny, nz = grid
    N, Q = z.shape
    Z = z.reshape(nz, ny, nx, Q)
    out = np.zeros_like(Z)
    for axis in range(3):
        if Z.shape[axis] < 2:
            continue
        diff = np.diff(Z, axis=axis)                  # z_{i+1} - z_i
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[axis] = slice(0, Z.shape[axis] - 1)
        hi[axis] = slice(1, Z.shape[axis])
        out[tuple(lo)] -= diff
        out[tuple(hi)] += diff
    return 2.0 * out.reshape(N, Q)


def reg_value(z: np.ndarray, grid) -> float:
    """R(z) = 1/2 ||D z||^2 = 1/2 <z, D^T D z> (Eq. l2)."""
    return 0.5 * float(np.sum(z * dtd_apply(z, grid)))


def dtd_norm(grid, dense_limit: int = 1024) -> float:
    """Spectral norm ||D^T D||_2.

    Small grids: largest eigenvalue of the dense D^T D (built by applying the
    operator to the identity). Larger grids: D^T D = 2 (L_x (+) L_y (+) L_z),
    a Kronecker sum of path-graph Laplacians whose largest eigenvalues are
    2 + 2 cos(pi / n_a) (0 for a single-voxel axis)."""
    nx, ny, nz = grid
    N = nx * ny * nz
    if N <= dense_limit:
        A = dtd_apply(np.eye(N), grid)
        return float(np.linalg.eigvalsh(0.5 * (A + A.T))[-1])
    lam = 0.0
    for n in (nx, ny, nz):
        if n > 1:
            lam += 2.0 + 2.0 * np.cos(np.pi / n)
    return 2.0 * lam


def xi_rule(lam: float, grid) -> float:
    """xi_p = 0.75 lambda ||D^T D|| + epsilon (Eq. sigma_cond)."""
    return XI_FACTOR * lam * dtd_norm(grid) + EPS_XI


# --------------------------------------------------------------- masked voxel sets
# Sec. II-C (maskless footnote): only voxels inside the object are estimated,
# with no smoothness across the object boundary. The regulariser of Eq. (l2)
# then runs over the face-neighbour pairs whose two voxels are both inside,
# i.e. over the graph induced by the mask; outside voxels stay 0.
def graph_edges(grid, mask):
    """Face-neighbour pairs (a, b), a < b, of inside voxels, as indices into
    the list of inside voxels (in increasing voxel order)."""
    nx, ny, nz = grid
    inside = np.asarray(mask, dtype=bool).reshape(-1)
    comp = -np.ones(inside.size, dtype=np.int64)
    comp[inside] = np.arange(int(inside.sum()))
    edges = []
    for n in np.flatnonzero(inside):
        x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
        for dx, dy, dz, lim, c in ((1, 0, 0, nx, x), (0, 1, 0, ny, y), (0, 0, 1, nz, z)):
            if c + 1 < lim:
                m = n + dx + nx * (dy + ny * dz)
                if inside[m]:
                    edges.append((comp[n], comp[m]))
    return np.asarray(edges, dtype=np.int64).reshape(-1, 2)


def dtd_apply_graph(z: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """D^T D z on an edge list: each pair (a, b) adds 2 (z_a - z_b) to a and
    2 (z_b - z_a) to b (each unordered pair is two ordered pairs of Eq. l2)."""
    out = np.zeros_like(z)
    if len(edges):
        a, b = edges[:, 0], edges[:, 1]
        diff = z[a] - z[b]
        np.add.at(out, a, 2.0 * diff)
        np.add.at(out, b, -2.0 * diff)
    return out


def dtd_norm_graph(edges: np.ndarray, n: int, dense_limit: int = 2048) -> float:
    """||D^T D||_2 on an edge list: dense eigvalsh up to dense_limit vertices,
    else ARPACK (scipy eigsh) on the sparse matrix."""
    if n <= dense_limit:
        A = dtd_apply_graph(np.eye(n), edges)
        return float(np.linalg.eigvalsh(0.5 * (A + A.T))[-1])
    import scipy.sparse as sp
    from scipy.sparse.linalg import eigsh
    a, b = edges[:, 0], edges[:, 1]
    deg = np.bincount(np.concatenate([a, b]), minlength=n).astype(np.float64)
    L = sp.coo_matrix((np.concatenate([deg, -np.ones(2 * len(a))]),
                       (np.concatenate([np.arange(n), a, b]),
                        np.concatenate([np.arange(n), b, a]))), shape=(n, n)).tocsr()
    return float(2.0 * eigsh(L, k=1, which="LA", return_eigenvectors=False)[0])


# --------------------------------------------------------------- objective
def objective(K_r: np.ndarray, m: np.ndarray, z: np.ndarray, grid, lam: float) -> float:
    """Cost of Eq. (spat) with R of Eq. (l2): 1/2 ||m - (I (x) K_r) z||^2 + lambda R(z)."""
    res = m - z @ K_r.T
    return 0.5 * float(np.sum(res * res)) + lam * reg_value(z, grid)


# --------------------------------------------------------------- LADMM steps
def f_step(c: np.ndarray, V_r: np.ndarray, s_w: np.ndarray, beta: float) -> np.ndarray:
    """f_n = c_n / beta - sum_i s_i v_i (v_i^T c_n) for every voxel (Eq. DictVecSVD)."""
    return c / beta - ((c @ V_r) * s_w) @ V_r.T


def z_step(z, f, d, lam, xi, beta, grid):
    """z^{k+1} = max(0, (xi z - lambda D^T D z + beta f + d) / (xi + beta)) (Eq. z2)."""
    return np.maximum(0.0, (xi * z - lam * dtd_apply(z, grid) + beta * f + d) / (xi + beta))


def d_step(d, z_new, f, beta):
    """d^{k+1} = d^k - beta (z^{k+1} - f^{k+1}) (dual update)."""
    return d - beta * (z_new - f)


def ladmm(K, m, grid, lam, beta, iters, rank=0, xi=None, z0=None, d0=None,
          track_every=0, f_star=None, mask=None, stop_tol=0.0, check_every=0):
    """Run Algorithm 2 for a fixed number of iterations.

    Returns a dict with z, f, d (N, Q), the rank r, xi and, when
    track_every > 0, a history of (k, objective(z^k), DFCS(z^k)) where DFCS
    follows Eq. (DFCS) against f_star when one is given, and beside it
    hist_f of (k, ||z^k - f^k||, DFCS(f^k)) -- the primal residual of the
    splitting f = z and the distance of f^k itself (f^0 = 0).

    mask (N booleans, optional): estimate the inside voxels only, on the graph
    of inside face neighbours (see graph_edges); outside voxels stay 0 and
    their data is ignored. stop_tol > 0 with check_every > 0: stop after
    iteration k+1 when k+1 is a multiple of check_every and
    ||z^{k+1} - z^k|| <= stop_tol ||z^{k+1}|| (the relative change of the
    iterate; "iters" returned is the number run)."""
    if mask is not None:
        return _ladmm_masked(K, m, grid, lam, beta, iters, rank, xi, mask, stop_tol, check_every)
    K = np.asarray(K, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    nx, ny, nz = grid
    N = nx * ny * nz
    P, Q = K.shape
    if m.shape != (N, P):
        raise ValueError("m must be (N, P)")
    U, s, V = thin_svd(K)
    r = rank_rule(s, rank)
    U_r, s_r, V_r = U[:, :r], s[:r], V[:, :r]
    if xi is None:
        xi = xi_rule(lam, grid)
    # weights sigma_i^2 / (beta^2 + beta sigma_i^2) of Eq. (DictVecSVD)
    s_w = s_r * s_r / (beta * beta + beta * s_r * s_r)
    # g_n = sum_{i<=r} sigma_i v_i u_i^T m_n
    g = ((m @ U_r) * s_r) @ V_r.T
    z = np.zeros((N, Q)) if z0 is None else np.array(z0, dtype=np.float64)
    d = np.zeros((N, Q)) if d0 is None else np.array(d0, dtype=np.float64)
    f = np.zeros((N, Q))
    K_r = (U_r * s_r) @ V_r.T
    hist, hist_f = [], []
    run = iters
    for k in range(iters):
        if track_every and k % track_every == 0:
            hist.append(_track(k, K_r, m, z, grid, lam, f_star))
            hist_f.append(_track_f(k, z, f, f_star))
        c = g + beta * z - d
        f = f_step(c, V_r, s_w, beta)
        z_new = z_step(z, f, d, lam, xi, beta, grid)
        d = d_step(d, z_new, f, beta)
        stop = _converged(z, z_new, k, stop_tol, check_every)
        z = z_new
        if stop:
            run = k + 1
            break
    if track_every:
        hist.append(_track(run, K_r, m, z, grid, lam, f_star))
        hist_f.append(_track_f(run, z, f, f_star))
    return dict(z=z, f=f, d=d, rank=r, xi=float(xi), sigma=s, hist=hist, hist_f=hist_f, K_r=K_r,
                iters=run)


def _converged(z, z_new, k, stop_tol, check_every):
    """Residual stopping rule: relative change of the iterate at a check."""
    if not (stop_tol > 0 and check_every > 0) or (k + 1) % check_every:
        return False
    return float(np.linalg.norm(z_new - z)) <= stop_tol * float(np.linalg.norm(z_new))


def _ladmm_masked(K, m, grid, lam, beta, iters, rank, xi, mask, stop_tol, check_every):
    """Algorithm 2 on the inside voxels only (graph regulariser), scattered
    back to the full grid with zeros outside."""
    K = np.asarray(K, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    nx, ny, nz = grid
    N = nx * ny * nz
    P, Q = K.shape
    inside = np.asarray(mask, dtype=bool).reshape(-1)
    if inside.size != N or m.shape != (N, P):
        raise ValueError("mask must have N entries and m must be (N, P)")
    idx = np.flatnonzero(inside)
    edges = graph_edges(grid, inside)
    n_in = idx.size
    U, s, V = thin_svd(K)
    r = rank_rule(s, rank)
    U_r, s_r, V_r = U[:, :r], s[:r], V[:, :r]
    if xi is None:
        xi = XI_FACTOR * lam * dtd_norm_graph(edges, n_in) + EPS_XI
    s_w = s_r * s_r / (beta * beta + beta * s_r * s_r)
    g = ((m[idx] @ U_r) * s_r) @ V_r.T
    z = np.zeros((n_in, Q))
    d = np.zeros((n_in, Q))
    f = np.zeros((n_in, Q))
    run = iters
    for k in range(iters):
        c = g + beta * z - d
        f = f_step(c, V_r, s_w, beta)
        z_new = np.maximum(0.0, (xi * z - lam * dtd_apply_graph(z, edges) + beta * f + d) /
                           (xi + beta))
        d = d_step(d, z_new, f, beta)
        stop = _converged(z, z_new, k, stop_tol, check_every)
        z = z_new
        if stop:
            run = k + 1
            break
    out = {}
    for name, a in (("z", z), ("f", f), ("d", d)):
        full = np.zeros((N, Q))
        full[idx] = a
        out[name] = full
    K_r = (U_r * s_r) @ V_r.T
    out.update(rank=r, xi=float(xi), sigma=s, hist=[], K_r=K_r, iters=run, edges=edges, inside=idx)
    return out


def objective_masked(K_r, m, z, grid, lam, mask) -> float:
    """Eq. (spat) over the inside voxels with the graph regulariser."""
    inside = np.asarray(mask, dtype=bool).reshape(-1)
    idx = np.flatnonzero(inside)
    edges = graph_edges(grid, inside)
    zi = z[idx]
    res = m[idx] - zi @ K_r.T
    return 0.5 * float(np.sum(res * res)) + lam * 0.5 * float(np.sum(zi * dtd_apply_graph(zi, edges)))


# --------------------------------------------------------------- penalty heuristic
def centre_patch(grid, size=3):
    """The size^d sub-box at the centre of the grid (d = axes longer than 1),
    clipped to the grid: (origin, patch grid)."""
    org, dims = [], []
    for n in grid:
        w = min(size, n)
        org.append((n - w) // 2)
        dims.append(w)
    return tuple(org), tuple(dims)


def patch_data(m, grid, origin, pgrid):
    """Rows of m (voxel-major) of the sub-box origin + pgrid, in the patch's voxel order."""
    nx, ny, _ = grid
    rows = []
    for zz in range(pgrid[2]):
        for yy in range(pgrid[1]):
            for xx in range(pgrid[0]):
                rows.append((origin[0] + xx) + nx * ((origin[1] + yy) + ny * (origin[2] + zz)))
    return m[np.asarray(rows)]


def beta_heuristic(K, m, grid, lam, iters, betas, rank=0, size=3):
    """Penalty selection of Sec. III-F: solve the centre patch (3 x 3, or
    3 x 3 x 3 in 3-D) for `iters` iterations at every candidate beta and keep
    the beta whose iterate has the lowest objective of Eq. (spat) on the patch
    (the fastest progress within the iteration budget). Returns
    (best beta, objectives)."""
    origin, pgrid = centre_patch(grid, size)
    mp = patch_data(np.asarray(m, dtype=np.float64), grid, origin, pgrid)
    J = []
    for b in betas:
        out = ladmm(K, mp, pgrid, lam, float(b), iters, rank=rank)
        J.append(objective(out["K_r"], mp, out["z"], pgrid, lam))
    J = np.asarray(J)
    return float(betas[int(np.argmin(J))]), J


def _track_f(k, z, f, f_star):
    """Primal residual ||z^k - f^k|| of the constraint f = z, and DFCS(f^k)."""
    dfcs = None
    if f_star is not None:
        dfcs = float(np.linalg.norm(f - f_star) / np.linalg.norm(f_star))
    return (k, float(np.linalg.norm(z - f)), dfcs)


def _track(k, K_r, m, z, grid, lam, f_star):
    J = objective(K_r, m, z, grid, lam)
    dfcs = None
    if f_star is not None:
        dfcs = float(np.linalg.norm(z - f_star) / np.linalg.norm(f_star))
    return (k, J, dfcs)
