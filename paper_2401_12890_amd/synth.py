"""Seeded synthetic mapping problems (dictionary K, voxel data m, box grid).

This module only draws inputs. It holds none of the LADMM arithmetic, so both
the HIP path and the FP64 oracle can be fed from it without sharing any of the
method's code.

The paper's datasets (DR-CSI, IR-MSE, MSE-T2, MRF; Sec. IV) are not available,
so every workload is a synthetic stand-in with the same structure: a
multi-exponential (or inversion-recovery fingerprinting) dictionary on a
log-spaced 2-D spectral grid, a nonnegative spectroscopic image made of a few
spectral blobs whose weights vary smoothly in space, and Gaussian noise
(the linear mixture model m_n = K f_n + noise of Sec. II-A).

Index conventions (shared with the library's C ABI):
  * voxel n = x + nx*(y + ny*z) on an (nx, ny, nz) box grid;
  * spectral node q = i1*n2 + i2 (first spectral axis major);
  * measurement p = i_b*n_TE + i_TE for diffusion-relaxation dictionaries;
  * m is voxel-major: m[n, p].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Workload recipes. Sizes follow the paper's kinds of experiment (Sec. IV);
# the numbers themselves are this project's synthetic choices.
CONFIGS = {
    # 2-D diffusion-relaxation, FP64 path
    "c1": dict(kind="dr", grid=(32, 32, 1), b=(0, 500, 1000, 2000, 3000),
               te=tuple(np.linspace(50.0, 150.0, 6)), n1=10, n2=10,
               ax1=(1e-4, 3e-3), ax2=(10.0, 2000.0), snr=100.0, lam=1e-2,
               iters=500, precision="fp64", seed=1, beta=0.1),
    # 3-D diffusion-relaxation, FP32 path
    "c2": dict(kind="dr", grid=(128, 128, 64), b=(0, 500, 1000, 1500, 2000, 3000),
               te=tuple(np.linspace(50.0, 150.0, 10)), n1=40, n2=40,
               ax1=(1e-4, 3e-3), ax2=(10.0, 2000.0), snr=50.0, lam=1e-2,
               iters=300, precision="fp32", seed=2, beta=0.1),
    # 3-D T1-T2 fingerprinting-like, split-precision path
    "c3": dict(kind="irfp", grid=(96, 96, 32), P=1000, n1=32, n2=32,
               ax1=(100.0, 4000.0), ax2=(10.0, 2000.0), tr=10.0,
               flip=(5.0, 60.0), te_range=(2.0, 100.0), snr=50.0, lam=1e-2,
               iters=300, precision="bf16x3", seed=3, beta=0.1),
}


@dataclass
class Problem:
    """One synthetic mapping problem."""
    K: np.ndarray              # (P, Q) float64, row-major
    m: np.ndarray              # (N, P) float64, voxel-major
    grid: tuple                # (nx, ny, nz)
    lam: float
    beta: float
    iters: int
    precision: str
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        nx, ny, nz = self.grid
        return nx * ny * nz

    @property
    def P(self) -> int:
        return self.K.shape[0]

    @property
    def Q(self) -> int:
        return self.K.shape[1]


def _logspace(lo, hi, n):
    return np.logspace(np.log10(lo), np.log10(hi), n)


def dictionary(cfg: dict, rng: np.random.Generator) -> tuple[np.ndarray, dict]:
    """Dictionary K (P x Q) for a recipe; unit quadrature weights."""
    a1 = _logspace(*cfg["ax1"], cfg["n1"])
    a2 = _logspace(*cfg["ax2"], cfg["n2"])
    g1 = np.repeat(a1, cfg["n2"])          # q = i1*n2 + i2
    g2 = np.tile(a2, cfg["n1"])
    if cfg["kind"] == "dr":
        b = np.asarray(cfg["b"], dtype=np.float64)
        te = np.asarray(cfg["te"], dtype=np.float64)
        bp = np.repeat(b, te.size)         # p = i_b*n_TE + i_TE
        tep = np.tile(te, b.size)
        K = np.exp(-np.outer(bp, g1)) * np.exp(-np.outer(tep, 1.0 / g2))
        meta = dict(b=bp, te=tep)
    elif cfg["kind"] == "irfp":
        P = cfg["P"]
        alpha = np.deg2rad(rng.uniform(cfg["flip"][0], cfg["flip"][1], P))
        te = rng.uniform(cfg["te_range"][0], cfg["te_range"][1], P)
        e1 = np.exp(-cfg["tr"] / g1)       # per spectral node (T1 axis)
        mz = -np.ones_like(g1)             # after inversion
        K = np.empty((P, g1.size))
        for p in range(P):
            K[p] = mz * np.sin(alpha[p]) * np.exp(-te[p] / g2)
            mz = mz * np.cos(alpha[p]) * e1 + (1.0 - e1)
        meta = dict(alpha=alpha, te=te)
    else:
        raise ValueError(cfg["kind"])
    meta.update(ax1=a1, ax2=a2)
    return K, meta


def _blobs(cfg, rng, nblob=3):
    l1 = np.log10(np.asarray(cfg["ax1"], dtype=np.float64))
    l2 = np.log10(np.asarray(cfg["ax2"], dtype=np.float64))
    x1 = np.repeat(np.linspace(l1[0], l1[1], cfg["n1"]), cfg["n2"])
    x2 = np.tile(np.linspace(l2[0], l2[1], cfg["n2"]), cfg["n1"])
    G = np.empty((nblob, x1.size))
    for j in range(nblob):
        c1 = l1[0] + (0.2 + 0.6 * rng.uniform()) * (l1[1] - l1[0])
        c2 = l2[0] + (0.2 + 0.6 * rng.uniform()) * (l2[1] - l2[0])
        w = rng.uniform(0.08, 0.20)
        g = np.exp(-((x1 - c1) ** 2 + (x2 - c2) ** 2) / (2.0 * w * w))
        G[j] = g / g.sum()
    return G


def _fields(grid, rng, nblob=3, nbump=6):
    """Smooth nonnegative weights a_j(r) >= 0.05 on the grid, shape (nblob, N)."""
    nx, ny, nz = grid
    dims = [(nx, 0), (ny, 1), (nz, 2)]
    coords = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = [coords[2].ravel().astype(np.float64), coords[1].ravel().astype(np.float64),
           coords[0].ravel().astype(np.float64)]
    A = np.empty((nblob, nx * ny * nz))
    for j in range(nblob):
        acc = np.full(nx * ny * nz, 0.05)
        for _ in range(nbump):
            amp = rng.uniform(0.2, 1.0)
            s = rng.uniform(0.1, 0.3)
            c = rng.uniform(0.0, 1.0, 3)
            r2 = np.zeros(nx * ny * nz)
            for (n, ax) in dims:
                if n > 1:
                    r2 += ((pos[ax] - c[ax] * n) / (s * n)) ** 2
            acc += amp * np.exp(-0.5 * r2)
        A[j] = acc
    return A


def generate(name: str, grid=None, seed=None, iters=None, overrides=None, dict_seed=None,
             single=False) -> Problem:
    """Seeded problem for recipe `name`, optionally on another grid or seed.

    Streams (spawned from SeedSequence(seed) in this order): dictionary
    parameters, spectral blobs, spatial fields, noise. `overrides` replaces
    recipe entries; `dict_seed` draws the dictionary parameters from that seed
    instead (jobs sharing one acquisition protocol share one dictionary);
    `single` forms the data and draws the noise in float32 (m is float32 then),
    for large served jobs; the float32 noise is a different seeded stream.
    """
    cfg = dict(CONFIGS[name])
    if overrides:
        cfg.update(overrides)
    if grid is not None:
        cfg["grid"] = tuple(int(v) for v in grid)
    if seed is None:
        seed = cfg["seed"]
    ss = np.random.SeedSequence(seed)
    r_dict, r_blob, r_field, r_noise = [np.random.Generator(np.random.PCG64(s))
                                        for s in ss.spawn(4)]
    if dict_seed is not None:
        r_dict = np.random.Generator(np.random.PCG64(np.random.SeedSequence(dict_seed).spawn(4)[0]))
    K, meta = dictionary(cfg, r_dict)
    G = _blobs(cfg, r_blob)                   # (3, Q)
    A = _fields(cfg["grid"], r_field)         # (3, N)
    KG = G @ K.T                              # (3, P): K applied to each blob
    if single:
        m = A.T.astype(np.float32) @ KG.astype(np.float32)
    else:
        m = A.T @ KG                          # (N, P) noise-free data
    if cfg["kind"] == "dr":
        p0 = 0                                # b = 0, shortest TE
    else:
        p0 = int(np.argmax(np.abs(m).mean(axis=0)))
    sigma = float(np.abs(m[:, p0]).mean()) / cfg["snr"]
    if single:
        m += np.float32(sigma) * r_noise.standard_normal(m.shape, dtype=np.float32)
    else:
        m += sigma * r_noise.standard_normal(m.shape)
    meta.update(sigma=sigma, p0=p0, blobs=G, fields=A, name=name, seed=seed)
    return Problem(K=K, m=m, grid=cfg["grid"], lam=cfg["lam"], beta=cfg["beta"],
                   iters=cfg["iters"] if iters is None else iters,
                   precision=cfg["precision"], meta=meta)


def random_problem(P, Q, grid, seed, lam=1e-2, beta=1.0, positive_K=False,
                   noise=0.01) -> Problem:
    """Small generic problem (random dictionary) for edge cases and pins."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if positive_K:
        K = rng.uniform(0.0, 1.0, (P, Q))
    else:
        K = rng.standard_normal((P, Q))
    nx, ny, nz = grid
    N = nx * ny * nz
    f = np.abs(rng.standard_normal((N, Q)))
    m = f @ K.T + noise * rng.standard_normal((N, P))
    return Problem(K=K, m=m, grid=(nx, ny, nz), lam=lam, beta=beta, iters=50,
                   precision="fp64", meta=dict(seed=seed))


# Batched uneven slices: 64 2-D slices with sides U{48..256}, P in {30, 60},
# Q in {100, 400, 1600} diffusion-relaxation dictionaries.
BATCH_C4 = dict(nslices=64, side=(48, 256), P=(30, 60), grid_n=(10, 20, 40), snr=50.0,
                lam=1e-2, beta=0.1, iters=200, seed=4)


def generate_batch(nslices=None, side=None, seed=None, iters=None, max_side=None):
    """Seeded list of Problems for the batched workload (each slice has its
    own grid, dictionary and data). The per-slice shape draws come from
    their own stream, so changing the sizes does not reshuffle the data."""
    cfg = dict(BATCH_C4)
    if nslices is not None:
        cfg["nslices"] = nslices
    if side is not None:
        cfg["side"] = side
    if seed is None:
        seed = cfg["seed"]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed).spawn(1)[0]))
    probs = []
    for k in range(cfg["nslices"]):
        nx = int(rng.integers(cfg["side"][0], cfg["side"][1] + 1))
        ny = int(rng.integers(cfg["side"][0], cfg["side"][1] + 1))
        if max_side is not None:
            nx, ny = min(nx, max_side), min(ny, max_side)
        P = int(rng.choice(cfg["P"]))
        n = int(rng.choice(cfg["grid_n"]))
        over = dict(n1=n, n2=n, snr=cfg["snr"], lam=cfg["lam"], beta=cfg["beta"],
                    iters=cfg["iters"] if iters is None else iters, precision="fp32")
        pr = generate("c1" if P == 30 else "c2", grid=(nx, ny, 1), seed=1000 * seed + k,
                      overrides=over)
        pr.meta["slice"] = k
        probs.append(pr)
    return probs


# Served stream: Poisson arrivals at `rate` jobs/s; N log-uniform on
# [1e3, 1e6] voxels, planar (nz = 1) up to 65,536 voxels, else volumetric with
# nz = 32; the dictionary class Q in {100, 400, 1024, 1600} uniform, each
# taking P, precision and iteration count from its recipe. Jobs of one class
# share one dictionary (one acquisition protocol).
SERVE_C5 = dict(rate=20.0, njobs=60, N=(1e3, 1e6), planar_max=65536, nz=32, seed=5,
                classes={100: ("c1", {}), 400: ("c2", dict(n1=20, n2=20)),
                         1024: ("c3", {}), 1600: ("c2", {})})


def _box(N, planar_max, nz):
    if N <= planar_max:
        nx = max(1, int(round(np.sqrt(N))))
        return (nx, max(1, int(round(N / nx))), 1)
    nx = max(1, int(round(np.sqrt(N / nz))))
    return (nx, max(1, int(round(N / (nz * nx)))), nz)


def serving_stream(njobs=None, rate=None, seed=None, N=None):
    """Seeded job specs of the served stream (no data): a list of dicts with
    the arrival time t (s), Q, the recipe name and overrides, the grid and
    the data seed. Times, sizes and classes come from one stream in job order."""
    cfg = dict(SERVE_C5)
    njobs = cfg["njobs"] if njobs is None else njobs
    rate = cfg["rate"] if rate is None else rate
    seed = cfg["seed"] if seed is None else seed
    lo, hi = cfg["N"] if N is None else N
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed).spawn(1)[0]))
    gaps = rng.exponential(1.0 / rate, njobs)
    t = np.cumsum(gaps) - gaps[0]
    Qs = sorted(cfg["classes"])
    specs = []
    for k in range(njobs):
        n = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        Q = int(Qs[rng.integers(len(Qs))])
        name, over = cfg["classes"][Q]
        specs.append(dict(t=float(t[k]), Q=Q, recipe=name, overrides=dict(over),
                          grid=_box(n, cfg["planar_max"], cfg["nz"]), seed=1000 * seed + k))
    return specs


def serving_problem(spec, single=True) -> Problem:
    """The Problem of one served job (dictionary from its recipe's own seed)."""
    name = spec["recipe"]
    return generate(name, grid=spec["grid"], seed=spec["seed"], overrides=spec["overrides"],
                    dict_seed=CONFIGS[name]["seed"], single=single)
