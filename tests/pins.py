"""Independent reference routines that pin the FP64 oracle.

None of these re-types the oracle's formulas: each reaches the same quantity
by a different route (definition by loops, exhaustive enumeration, a
different solver, a dense linear system), so a dropped term, a wrong sign or
index, or a transposed operand in the oracle shows up as a disagreement.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def voxel_index(x, y, z, grid):
    nx, ny, _ = grid
    return x + nx * (y + ny * z)


def neighbours(n, grid):
    """Face neighbours Delta(n) of voxel n on the box grid (free boundary)."""
    nx, ny, nz = grid
    x = n % nx
    y = (n // nx) % ny
    z = n // (nx * ny)
    out = []
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        a, b, c = x + dx, y + dy, z + dz
        if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
            out.append(voxel_index(a, b, c, grid))
    return out


def explicit_D(grid):
    """Sparse D with one row e_n - e_m per ordered adjacent pair (n, m), so that
    1/2 ||D f||^2 equals sum_n sum_{m in Delta(n)} 1/2 ||f_n - f_m||^2 (Eq. l2)."""
    nx, ny, nz = grid
    N = nx * ny * nz
    rows, cols, vals = [], [], []
    k = 0
    for n in range(N):
        for m in neighbours(n, grid):
            rows += [k, k]
            cols += [n, m]
            vals += [1.0, -1.0]
            k += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(k, N))


def explicit_D_masked(grid, mask):
    """Sparse D over the inside voxels only (columns: inside voxels in increasing
    voxel order), one row per ordered pair of inside face neighbours."""
    inside = np.asarray(mask, dtype=bool).reshape(-1)
    idx = np.flatnonzero(inside)
    col = {int(n): c for c, n in enumerate(idx)}
    rows, cols, vals = [], [], []
    k = 0
    for n in idx:
        for m in neighbours(int(n), grid):
            if inside[m]:
                rows += [k, k]
                cols += [col[int(n)], col[m]]
                vals += [1.0, -1.0]
                k += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(k, len(idx)))


def R_loops(f, grid):
    """R(f) by the double sum of Eq. (l2), with plain loops."""
    N = f.shape[0]
    total = 0.0
    for n in range(N):
        for m in neighbours(n, grid):
            diff = f[n] - f[m]
            total += 0.5 * float(diff @ diff)
    return total


def nnls_bruteforce(K, m):
    """argmin_{f>=0} 1/2 ||m - K f||^2 by enumerating every support (tiny Q).

    For full-column-rank K the minimiser is unique; on each support the
    unconstrained least-squares solution is computed, and the feasible one that
    also satisfies the KKT sign condition on the complement is returned."""
    P, Q = K.shape
    best, best_J = None, np.inf
    for size in range(0, Q + 1):
        for S in itertools.combinations(range(Q), size):
            f = np.zeros(Q)
            if size:
                KS = K[:, S]
                sol, *_ = np.linalg.lstsq(KS, m, rcond=None)
                if np.any(sol < 0):
                    continue
                f[list(S)] = sol
            J = 0.5 * float(np.sum((m - K @ f) ** 2))
            if J < best_J - 1e-15:
                best, best_J = f, J
    return best


def dense_problem_matrices(K_r, m, grid, lam):
    """Normal-equation matrix and right side of the unconstrained version of
    Eq. (spat): (I (x) K^T K + lam D^T D (x) I) f = (I (x) K^T) m, voxel-major."""
    D = explicit_D(grid).toarray()
    N = D.shape[1]
    P, Q = K_r.shape
    A = np.kron(np.eye(N), K_r.T @ K_r) + lam * np.kron(D.T @ D, np.eye(Q))
    rhs = (m @ K_r).reshape(-1)
    return A, rhs


def interior_solution(K_r, m, grid, lam):
    A, rhs = dense_problem_matrices(K_r, m, grid, lam)
    f = np.linalg.solve(A, rhs)
    return f.reshape(m.shape[0], K_r.shape[1])


def grad_J(K_r, m, z, grid, lam):
    """Gradient of 1/2||m - (I(x)K_r) z||^2 + lam/2 ||D z||^2 using the explicit D."""
    D = explicit_D(grid)
    DtD = (D.T @ D).tocsr()
    return (z @ K_r.T - m) @ K_r + lam * (DtD @ z)


def J_explicit(K_r, m, z, grid, lam):
    res = m - z @ K_r.T
    D = explicit_D(grid)
    Dz = D @ z
    return 0.5 * float(np.sum(res * res)) + lam * 0.5 * float(np.sum(Dz * Dz))


def fista(K_r, m, grid, lam, iters=20000, tol=1e-14, D=None):
    """Projected gradient with Nesterov momentum and adaptive restart on the
    same convex problem, using the explicit sparse D (independent of LADMM);
    D may be given (e.g. a masked one over a subset of voxels, with m's rows)."""
    if D is None:
        D = explicit_D(grid)
    DtD = (D.T @ D).tocsr()
    Lip = np.linalg.norm(K_r, 2) ** 2 + lam * np.linalg.norm(DtD.toarray(), 2)
    step = 1.0 / Lip
    N, Q = m.shape[0], K_r.shape[1]
    x = np.zeros((N, Q))
    y = x.copy()
    t = 1.0

    def J(v):
        res = m - v @ K_r.T
        Dv = D @ v
        return 0.5 * float(np.sum(res * res)) + 0.5 * lam * float(np.sum(Dv * Dv))

    Jx = J(x)
    for _ in range(iters):
        g = (y @ K_r.T - m) @ K_r + lam * (DtD @ y)
        x_new = np.maximum(0.0, y - step * g)
        J_new = J(x_new)
        if J_new > Jx:            # restart the momentum
            t = 1.0
            y = x.copy()
            continue
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        y = x_new + ((t - 1.0) / t_new) * (x_new - x)
        if abs(Jx - J_new) <= tol * max(1.0, abs(J_new)) and np.max(np.abs(x_new - x)) < 1e-13:
            x, Jx = x_new, J_new
            break
        x, Jx, t = x_new, J_new, t_new
    return x, Jx


def polish_active_set(K_r, m, z, grid, lam, thresh=1e-7):
    """Exact minimiser on the support of an approximate one: with the free set
    F = {z > thresh max z} and z = 0 elsewhere, solve the normal equations of the
    nonnegative problem restricted to F, H_FF z_F = b_F, with the dense Hessian
    H = I_N (x) K^T K + lambda D^T D (x) I_Q (explicit ordered-pair D, voxel-major
    z) and b = vec(K^T m_n). Returns (z, complementarity residual of the result);
    the support is right when the residual is at rounding level."""
    N, Q = z.shape
    D = explicit_D(grid)
    H = np.kron(np.eye(N), K_r.T @ K_r) + lam * np.kron((D.T @ D).toarray(), np.eye(Q))
    b = (m @ K_r).reshape(-1)
    F = np.flatnonzero(z.reshape(-1) > thresh * z.max())
    x = np.zeros(N * Q)
    x[F] = np.linalg.solve(H[np.ix_(F, F)], b[F])
    zp = x.reshape(N, Q)
    return zp, kkt_residual(K_r, m, zp, grid, lam)[1]


def kkt_residual(K_r, m, z, grid, lam):
    """Return (min z, max |min(z, grad)|-style complementarity, most negative
    gradient on the zero set) at z for the nonnegative problem."""
    g = grad_J(K_r, m, z, grid, lam)
    compl = np.max(np.abs(np.minimum(z, g)))     # zero iff z>=0, g>=0, z*g=0
    return float(z.min()), float(compl), float(g.min())
