"""FP64 CPU oracle: the previous ADMM of the paper (Algorithm 1, Sec. II-C).

TEST INFRASTRUCTURE ONLY (see the package docstring). The earlier approach
splits f three ways (data term x, nonnegativity y, regulariser z), each with
its own dual variable, so it keeps eight Q x N arrays (f, x, y, z, d_x, d_y,
d_z and g) against the three of Algorithm 2 (g, z, d). Its x-step applies
(K^T K + beta I)^{-1} with the full K, and its z-step inverts
lambda D^T D + beta I on each spectral plane. It serves as an independent
route to the same minimiser of Eq. (spat) (with K, i.e. Algorithm 2 at
r = min(P, Q)), not as a benchmark.

Same array conventions as algorithm2: (N, Q) voxel-major, box grid with
voxel n = x + nx*(y + ny*z), D^T D = 2 L with free ends.
"""
from __future__ import annotations

import numpy as np
from scipy.fft import dctn, idctn


def dtd_eigenvalues(grid) -> np.ndarray:
    """Eigenvalues of D^T D on the box with free ends, arranged like a
    (nz, ny, nx) plane: the DCT-II basis cos(pi k (j + 1/2) / n) diagonalises
    each path Laplacian with eigenvalue 2 - 2 cos(pi k / n), the Laplacian of
    the box is their Kronecker sum, and D^T D is twice it."""
    nx, ny, nz = grid
    ev = [2.0 - 2.0 * np.cos(np.pi * np.arange(n) / n) for n in (nz, ny, nx)]
    return 2.0 * (ev[0][:, None, None] + ev[1][None, :, None] + ev[2][None, None, :])


def z_solve_dct(b: np.ndarray, grid, lam: float, beta: float) -> np.ndarray:
    """(lambda D^T D + beta I)^{-1} b on every spectral plane, by the
    orthonormal 3-D DCT-II (the z-step of Algorithm 1)."""
    nx, ny, nz = grid
    N, Q = b.shape
    B = b.reshape(nz, ny, nx, Q)
    mu = dtd_eigenvalues(grid)[..., None]
    Bh = dctn(B, type=2, axes=(0, 1, 2), norm="ortho")
    return idctn(Bh / (lam * mu + beta), type=2, axes=(0, 1, 2), norm="ortho").reshape(N, Q)


def admm_previous(K, m, grid, lam, beta, iters, init=None):
    """Algorithm 1 for a fixed number of iterations, from zero initial values
    (as the algorithm states) or from `init`, a dict that may give any of
    f, x, y, z, dx, dy, dz as (N, Q) arrays (the rest start at zero).

    Returns the primal variables f, x, y, z and the duals d_x, d_y, d_z
    (all (N, Q)); y is the nonnegative iterate."""
    K = np.asarray(K, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    nx, ny, nz = grid
    N = nx * ny * nz
    P, Q = K.shape
    if m.shape != (N, P):
        raise ValueError("m must be (N, P)")
    Minv = np.linalg.inv(K.T @ K + beta * np.eye(Q))     # (K^T K + beta I)^{-1}
    g = m @ K                                           # g_n = K^T m_n
    init = init or {}
    start = {k: np.array(init[k], dtype=np.float64) if k in init else np.zeros((N, Q))
             for k in ("f", "x", "y", "z", "dx", "dy", "dz")}
    f, x, y, z = start["f"], start["x"], start["y"], start["z"]
    dx, dy, dz = start["dx"], start["dy"], start["dz"]
    for _ in range(iters):
        f = (beta * x + dx + beta * y + dy + beta * z + dz) / (3.0 * beta)
        x = (g + beta * f - dx) @ Minv.T
        y = np.maximum(0.0, f - dy / beta)
        z = z_solve_dct(beta * f - dz, grid, lam, beta)
        dx = dx - beta * (f - x)
        dy = dy - beta * (f - y)
        dz = dz - beta * (f - z)
    return dict(f=f, x=x, y=y, z=z, dx=dx, dy=dy, dz=dz)
