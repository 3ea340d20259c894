"""Batches: many problems of uneven size in shared fused launches.

Each job's map from the batch must be bitwise the map of the same job solved
alone (the per-voxel arithmetic does not depend on the brick shape or on the
other jobs in a launch), and within the precision's tolerance of the oracle.
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


@pytest.fixture(scope="module")
def slices():
    # the batched recipe at reduced sides so the oracle stays quick
    return synth.generate_batch(nslices=8, side=(17, 61), iters=30)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batch_equals_solo_and_oracle(torch_cuda, slices, prec):
    iters = 30
    say("batch", prec, [(p.grid, p.P, p.Q) for p in slices])
    with _ffi.BatchMapper([p.K for p in slices], [p.grid for p in slices]) as bm:
        F = bm.solve([p.m for p in slices], [p.lam for p in slices], [p.beta for p in slices],
                     iters, precision=prec)
        st = bm.stats()
    assert st["njobs"] == len(slices) and st["solo_jobs"] == 0
    assert sum(c["jobs"] for c in st["classes"]) == len(slices)
    for p, Fb in zip(slices, F):
        with _ffi.Mapper(p.K, p.grid) as mp:
            Fs = mp.solve(p.m, p.lam, p.beta, iters, precision=prec, kernel="fused")
        assert np.array_equal(Fb, Fs), p.grid
        ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, iters)
        err = np.linalg.norm(Fb - ref["z"]) / np.linalg.norm(ref["z"])
        assert err <= TOL[prec], (p.grid, p.Q, err)


def test_batch_persistent_walk_across_jobs(torch_cuda):
    # Volumetric float32 jobs with short spectra (3 and 4 chunks of 16 nodes) in one
    # class: 419 bricks of 16 x 8 x 4, more than the CUs, so each workgroup of the
    # persistent grid walks several bricks and its load stream crosses from one
    # job's bricks into the next job's. Ragged grids; Q = 36, 49, 64.
    iters = 10
    probs = [synth.generate("c2", grid=g, iters=iters, overrides=dict(n1=n, n2=n))
             for g, n in (((60, 62, 38), 6), ((40, 30, 21), 7), ((33, 17, 9), 8))]
    with _ffi.BatchMapper([p.K for p in probs], [p.grid for p in probs]) as bm:
        F = bm.solve([p.m for p in probs], [p.lam for p in probs], [p.beta for p in probs], iters,
                     precision="fp32")
        st = bm.stats()
    say("walk batch", st["classes"])
    assert st["nclasses"] == 1 and st["solo_jobs"] == 0
    assert st["classes"][0]["brick"] == (16, 8, 4) and st["classes"][0]["bricks"] == 419
    for p, Fb in zip(probs, F):
        with _ffi.Mapper(p.K, p.grid) as mp:
            Fs = mp.solve(p.m, p.lam, p.beta, iters, precision="fp32", kernel="fused")
        assert np.array_equal(Fb, Fs), p.grid
        ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, iters)
        err = np.linalg.norm(Fb - ref["z"]) / np.linalg.norm(ref["z"])
        assert err <= TOL["fp32"], (p.grid, p.Q, err)


def test_batch_autotune_keeps_the_bits(torch_cuda, slices):
    iters = 12
    with _ffi.BatchMapper([p.K for p in slices], [p.grid for p in slices]) as bm:
        args = ([p.m for p in slices], [p.lam for p in slices], [p.beta for p in slices], iters)
        F0 = bm.solve(*args, precision="fp32")
        F1 = bm.solve(*args, precision="fp32", autotune=True)
        st = bm.stats()
        # a later solve without the search keeps the shapes it chose
        F2 = bm.solve(*args, precision="fp32")
        st2 = bm.stats()
    assert st["autotune_ms"] > 0
    say("autotuned bricks", [c["brick"] for c in st["classes"]])
    assert [c["brick"] for c in st2["classes"]] == [c["brick"] for c in st["classes"]]
    for a, b, c in zip(F0, F1, F2):
        assert np.array_equal(a, b) and np.array_equal(a, c)


def test_batch_mixed_ranks_solo_jobs_and_device_entry(torch_cuda, slices):
    torch = torch_cuda
    iters = 10
    jobs = slices[:4]
    # job 1 at the unapproximated rank (min(P, Q) = 30 or 60: fused up to 32, else a solo job)
    ranks = [0, -1, 0, 7]
    with _ffi.BatchMapper([p.K for p in jobs], [p.grid for p in jobs]) as bm:
        steps = [_ffi.make_steps(p.beta, rank=r, precision="fp32") for p, r in zip(jobs, ranks)]
        Ms = [torch.tensor(p.m, dtype=torch.float32, device="cuda") for p in jobs]
        torch.cuda.synchronize()
        Fs = [torch.empty((p.N, p.Q), dtype=torch.float32, device="cuda") for p in jobs]
        s = torch.cuda.current_stream()
        _ffi.ssmap_batch_solve_device(bm.b, [M.data_ptr() for M in Ms], [p.lam for p in jobs],
                                      steps, iters, [F.data_ptr() for F in Fs], s.cuda_stream)
        torch.cuda.synchronize()
        st = bm.stats()
    say("classes", st["classes"], "solo", st["solo_jobs"])
    for p, r, F in zip(jobs, ranks, Fs):
        with _ffi.Mapper(p.K, p.grid) as mp:
            # a rank the fused kernel covers is compared with the fused kernel's solve
            kw = {} if r == -1 and min(p.P, p.Q) > 32 else {"kernel": "fused"}
            ref = mp.solve(p.m, p.lam, p.beta, iters, precision="fp32", rank=r, **kw)
        assert np.array_equal(F.cpu().numpy().astype(np.float64), ref)


def test_batch_errors(torch_cuda, slices):
    jobs = slices[:3]
    with _ffi.BatchMapper([p.K for p in jobs], [p.grid for p in jobs]) as bm:
        args = ([p.m for p in jobs], [p.lam for p in jobs], [p.beta for p in jobs], 3)
        with pytest.raises(_ffi.SsmapError) as e:
            bm.solve(*args, keep_aux=True)
        assert e.value.status == _ffi.SSMAP_EINVAL
        for kw in (dict(check_every=1, stop_tol=1e-3), dict(check_every=1, primal=True)):
            with pytest.raises(_ffi.SsmapError) as e:
                bm.solve(*args, **kw)
            assert e.value.status == _ffi.SSMAP_EINVAL, kw
        bad = [p.m.copy() for p in jobs]
        bad[2][0, 0] = np.inf
        with pytest.raises(_ffi.SsmapError) as e:
            bm.solve(bad, *args[1:])
        assert e.value.status == _ffi.SSMAP_ENONFINITE and "job 2" in str(e.value)
        F = bm.solve(*args, precision="fp32")
        assert all(np.isfinite(f).all() for f in F)


def disk_mask(grid, frac=0.35, seed=0):
    """A disk (planar) or ball of about `frac` of the box, off centre, with a hole."""
    nx, ny, nz = grid
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cx, cy, cz = 0.45 * nx, 0.55 * ny, 0.5 * (nz - 1)
    rr = ((x - cx) / nx) ** 2 + ((y - cy) / ny) ** 2 + (((z - cz) / nz) ** 2 if nz > 1 else 0)
    hole = ((x - cx) ** 2 + (y - cy) ** 2) < 2.5
    return ((rr < frac / 3.0) & ~hole).reshape(-1)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batch_with_masks_equals_masked_solo_and_oracle(torch_cuda, slices, prec):
    """Masks on some jobs of a batch (ssmap_batch_set_mask): each job's map equals
    its single masked solve bit for bit and the oracle's masked Algorithm 2; NaN
    data outside a mask is not read; the unmasked jobs are unchanged."""
    iters = 30
    jobs = slices[:5]
    masks = [disk_mask(p.grid) if j % 2 == 0 else None for j, p in enumerate(jobs)]
    Ms = []
    for p, mk in zip(jobs, masks):
        m = p.m.copy()
        if mk is not None:
            m[~mk] = np.nan
        Ms.append(m)
    with _ffi.BatchMapper([p.K for p in jobs], [p.grid for p in jobs]) as bm:
        for j, mk in enumerate(masks):
            if mk is not None:
                bm.set_mask(j, mk)
        F = bm.solve(Ms, [p.lam for p in jobs], [p.beta for p in jobs], iters, precision=prec)
        with pytest.raises(_ffi.SsmapError) as e:
            bm.set_mask(len(jobs), None)
        assert e.value.status == _ffi.SSMAP_EINVAL
    for p, mk, m, Fb in zip(jobs, masks, Ms, F):
        with _ffi.Mapper(p.K, p.grid) as mp:
            if mk is not None:
                mp.set_mask(mk)
            Fs = mp.solve(m, p.lam, p.beta, iters, precision=prec, kernel="fused")
        assert np.array_equal(Fb, Fs), p.grid
        ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, iters, mask=mk)
        err = np.linalg.norm(Fb - ref["z"]) / np.linalg.norm(ref["z"])
        say("masked batch", prec, p.grid, "inside", None if mk is None else int(mk.sum()), "err", err)
        assert err <= TOL[prec], (p.grid, err)
        if mk is not None:
            assert np.all(Fb[~mk] == 0.0)


def test_batch_monitoring_per_job(torch_cuda, slices):
    """check_every per job in a batch (ssmap_batch_get_job_stats): each monitored
    job's history equals its single solve's (objective and ||z|| to 1e-12; the
    dual residual to 1e-5, its per-brick float32 partial sums being grouped by
    the class's brick shape) and the oracle's objective within 1e-4; a job at
    the unapproximated rank runs outside the shared launches and is monitored
    on its own path; a job with check_every = 0 has no history."""
    iters = 20
    jobs = slices[:4]
    ranks = [-1, 0, 0, 0]            # job 0: P = 60, Q = 100, so r = 60, outside the fused classes
    every = [5, 10, 0, 4]
    steps = [_ffi.make_steps(p.beta, rank=r, precision="fp32", check_every=e)
             for p, r, e in zip(jobs, ranks, every)]
    with _ffi.BatchMapper([p.K for p in jobs], [p.grid for p in jobs]) as bm:
        F = _ffi.ssmap_batch_solve(bm.b, [p.m for p in jobs], [p.lam for p in jobs], steps, iters,
                                   [(p.N, p.Q) for p in jobs])
        sts = [bm.job_stats(j) for j in range(len(jobs))]
        with pytest.raises(_ffi.SsmapError):
            bm.job_stats(len(jobs))
    for p, r, e, st, Fb in zip(jobs, ranks, every, sts, F):
        if e == 0:
            assert st["hist_iter"] == []
            continue
        assert st["hist_iter"] == list(range(e, iters + 1, e))
        kw = {} if r == -1 and min(p.P, p.Q) > 32 else {"kernel": "fused"}
        with _ffi.Mapper(p.K, p.grid) as mp:
            Fs = mp.solve(p.m, p.lam, p.beta, iters, precision="fp32", rank=r, check_every=e, **kw)
            one = mp.stats()
        assert np.array_equal(Fb, Fs)
        ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, iters, rank=r, track_every=e)
        J = {k: v for (k, v, _) in ref["hist"]}
        say("monitored job", p.grid, "rank", st["rank"], "kernel", st["kernel"], "J", st["hist_objective"][-1])
        assert st["kernel"] == one["kernel"] and (r != -1 or st["kernel"] == 3)
        for i, k in enumerate(st["hist_iter"]):
            assert st["hist_objective"][i] == pytest.approx(one["hist_objective"][i], rel=1e-12)
            assert st["hist_znorm"][i] == pytest.approx(one["hist_znorm"][i], rel=1e-12)
            assert st["hist_dual"][i] == pytest.approx(one["hist_dual"][i], rel=1e-5)
            assert st["hist_objective"][i] == pytest.approx(J[k], rel=1e-4)
