"""Serving: jobs arriving over time, admitted under a device-memory budget and
advanced together in shared fused launches (continuous batching).

A served job's map must be bitwise the map of the same job solved alone with
the fused kernel (the per-voxel arithmetic does not depend on which other jobs
share a launch, on the round a job joins at, or on the stream), and within
the precision's tolerance of the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2401_12890_amd import _ffi, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5, "bf16x3": 1e-3}
TORCH_T = {"fp64": "float64", "fp32": "float32", "bf16x3": "float32"}


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
def jobs():
    """(problem, precision, iters): planar slices of the batched recipe plus
    volumetric crops of the three configuration generators, ragged sizes."""
    out = []
    for k, p in enumerate(synth.generate_batch(nslices=6, side=(17, 45), iters=25)):
        out.append((p, "fp32" if k % 2 == 0 else "bf16x3", 20 + 3 * k))
    out.append((synth.generate("c1", grid=(20, 13, 1)), "fp64", 31))
    out.append((synth.generate("c2", grid=(19, 11, 5)), "fp32", 17))
    out.append((synth.generate("c3", grid=(13, 9, 6)), "bf16x3", 14))
    out.append((synth.generate("c1", grid=(9, 7, 5)), "fp64", 22))
    return out


@pytest.fixture(scope="module")
def solo(torch_cuda, jobs):
    """Each job solved alone through the single-problem entry point."""
    torch = torch_cuda
    refs = []
    for p, prec, iters in jobs:
        M = torch.tensor(p.m, dtype=getattr(torch, TORCH_T[prec]), device="cuda")
        with _ffi.Mapper(p.K, p.grid) as mp:
            F = mp.solve_torch(M, p.lam, p.beta, iters, precision=prec, kernel="fused")
            torch.cuda.synchronize()
        refs.append(F)
    return refs


def device_inputs(torch, jobs):
    Ms = [torch.tensor(p.m, dtype=getattr(torch, TORCH_T[prec]), device="cuda")
          for p, prec, _ in jobs]
    torch.cuda.synchronize()
    return Ms


def serve(torch, jobs, budget, streams, stagger):
    """Submit the jobs (half, then the rest after a few pumps when staggered),
    drain, return the maps, the job infos and the server stats."""
    Ms = device_inputs(torch, jobs)
    with _ffi.Server(budget, streams) as sv:
        dict_of = {}
        ids = []
        for j, ((p, prec, iters), M) in enumerate(zip(jobs, Ms)):
            key = id(p.K)
            if key not in dict_of:
                dict_of[key] = sv.add_dictionary(p.K)
            ids.append(sv.submit(dict_of[key], p.grid, M, p.lam, p.beta, iters, ready=True,
                                 precision=prec))
            if stagger and j == len(jobs) // 2:
                for _ in range(3):
                    sv.pump(0.2)
        sv.drain()
        infos = [sv.poll(i) for i in ids]
        Fs = [sv.result(i) for i in ids]
        st = sv.stats()
    return Fs, infos, st


@pytest.mark.parametrize("streams,stagger", [(4, True), (1, False), (2, True)])
def test_served_jobs_equal_solo(torch_cuda, jobs, solo, streams, stagger):
    torch = torch_cuda
    say("serve", streams, stagger, [(p.grid, p.Q, prec, it) for p, prec, it in jobs])
    Fs, infos, st = serve(torch, jobs, 4e9, streams, stagger)
    assert st["completed"] == len(jobs) and st["submitted"] == len(jobs)
    assert st["in_use_bytes"] == 0 and st["peak_bytes"] <= st["budget_bytes"]
    for (p, prec, iters), F, ref, info in zip(jobs, Fs, solo, infos):
        assert info["state"] == "done" and info["status"] == _ffi.SSMAP_OK
        assert info["iters"] == iters
        assert info["submit_ms"] <= info["admit_ms"]
        assert torch.equal(F, ref), (p.grid, prec)


def test_served_jobs_match_oracle(torch_cuda, jobs, solo):
    torch = torch_cuda
    Fs, _, _ = serve(torch, jobs, 4e9, 4, True)
    for (p, prec, iters), F in zip(jobs, Fs):
        ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, iters)
        z = F.double().cpu().numpy()
        err = np.linalg.norm(z - ref["z"]) / np.linalg.norm(ref["z"])
        say("oracle", p.grid, prec, iters, err)
        assert err <= TOL[prec], (p.grid, prec, err)


def test_small_budget_queues_and_reuses_memory(torch_cuda, jobs, solo):
    torch = torch_cuda
    Ms = device_inputs(torch, jobs)
    # a budget that holds the largest job and little else: admission must wait
    # for retirements, and freed ranges are reused across streams
    with _ffi.Server(4e9, 4) as probe:
        sizes = []
        for (p, prec, iters), M in zip(jobs, Ms):
            d = probe.add_dictionary(p.K)
            jid = probe.submit(d, p.grid, M, p.lam, p.beta, 0, ready=True, precision=prec)
            sizes.append(probe.poll(jid)["state_bytes"])
        probe.drain()
    budget = 1.2 * max(sizes)
    say("budget", budget, "job bytes", sizes)
    Fs, infos, st = serve(torch, jobs, budget, 4, False)
    assert st["peak_bytes"] <= budget
    assert st["completed"] == len(jobs)
    for F, ref in zip(Fs, solo):
        assert torch.equal(F, ref)
    # strict arrival order: each job is admitted no earlier than the one before it
    admits = [i["admit_ms"] for i in infos]
    assert admits == sorted(admits)


def test_zero_iterations_nonfinite_and_rejections(torch_cuda, jobs):
    torch = torch_cuda
    p, prec, _ = jobs[0]
    M = torch.tensor(p.m, dtype=torch.float32, device="cuda")
    Mbad = M.clone()
    Mbad[3, 1] = float("nan")
    torch.cuda.synchronize()
    with _ffi.Server(1e9, 2) as sv:
        d = sv.add_dictionary(p.K)
        F0 = torch.full((p.N, p.Q), 7.0, device="cuda")
        j0 = sv.submit(d, p.grid, M, p.lam, p.beta, 0, F=F0, ready=True, precision="fp32")
        jb = sv.submit(d, p.grid, Mbad, p.lam, p.beta, 5, ready=True, precision="fp32")
        jg = sv.submit(d, p.grid, M, p.lam, p.beta, 5, ready=True, precision="fp32")
        bad = [dict(check_every=1, stop_tol=1e-3), dict(keep_aux=True), dict(autotune=True),
               dict(kernel="unfused"), dict(rank=p.K.shape[0] + 1)]
        for kw in bad:
            with pytest.raises(_ffi.SsmapError) as e:
                sv.submit(d, p.grid, M, p.lam, p.beta, 5, ready=True,
                          **dict(dict(precision="fp32"), **kw))
            assert e.value.status == _ffi.SSMAP_EINVAL, kw
        with pytest.raises(_ffi.SsmapError) as e:        # 33 monitor checks
            sv.submit(d, p.grid, M, p.lam, p.beta, 33, ready=True, precision="fp32", check_every=1)
        assert e.value.status == _ffi.SSMAP_EINVAL
        p2 = jobs[7][0]                                  # P = 60: rank 60 has no fused kernel
        d2 = sv.add_dictionary(p2.K)
        M2 = torch.tensor(p2.m, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(_ffi.SsmapError) as e:
            sv.submit(d2, p2.grid, M2, p2.lam, p2.beta, 5, ready=True, precision="fp32", rank=-1)
        assert e.value.status == _ffi.SSMAP_EINVAL
        with pytest.raises(_ffi.SsmapError) as e:        # alone above the budget
            _ffi.ssmap_server_submit(sv.sv, d, (2048, 2048, 1), M.data_ptr(), p.lam,
                                     _ffi.make_steps(p.beta, precision="fp32"), 5, M.data_ptr())
        assert e.value.status == _ffi.SSMAP_ENOMEM
        with pytest.raises(_ffi.SsmapError) as e:
            _ffi.ssmap_server_submit(sv.sv, 99, p.grid, M.data_ptr(), p.lam,
                                     _ffi.make_steps(p.beta, precision="fp32"), 5, M.data_ptr())
        assert e.value.status == _ffi.SSMAP_EINVAL
        sv.drain()
        assert sv.poll(j0)["state"] == "done"
        assert torch.count_nonzero(sv.result(j0)).item() == 0
        assert sv.poll(jb)["status"] == _ffi.SSMAP_ENONFINITE
        with pytest.raises(_ffi.SsmapError):
            sv.result(jb)
        assert sv.poll(jg)["status"] == _ffi.SSMAP_OK
        assert torch.isfinite(sv.result(jg)).all()
        with pytest.raises(_ffi.SsmapError):
            sv.poll(12345)


def test_served_jobs_monitored(torch_cuda, jobs):
    """check_every on served jobs (ssmap_server_get_job_stats): each monitored
    job's history equals the same job solved alone with the fused kernel and
    monitored alike (the same kernels, bricks and reductions over the same
    iterates), and its objective the oracle's; an unmonitored job in the same
    server has no history."""
    torch = torch_cuda
    sel = [jobs[0], jobs[1], jobs[6], jobs[8], jobs[9]]
    every = [5, 0, 7, 4, 3]
    Ms = device_inputs(torch, sel)
    with _ffi.Server(4e9, 4) as sv:
        ids = []
        for (p, prec, iters), M, e in zip(sel, Ms, every):
            d = sv.add_dictionary(p.K)
            ids.append(sv.submit(d, p.grid, M, p.lam, p.beta, iters, ready=True, precision=prec,
                                 check_every=e))
        sv.drain()
        sts = [sv.job_stats(i) for i in ids]
        Fs = [sv.result(i) for i in ids]
        with pytest.raises(_ffi.SsmapError):
            sv.job_stats(12345)
    J_TOL = {"fp64": 1e-9, "fp32": 1e-4, "bf16x3": 1e-3}
    for (p, prec, iters), e, st, F in zip(sel, every, sts, Fs):
        assert st["iters"] == iters and st["kernel"] == 2
        if e == 0:
            assert st["hist_iter"] == []
            continue
        expect = list(range(e, iters + 1, e)) + ([iters] if iters % e else [])
        assert st["hist_iter"] == expect
        with _ffi.Mapper(p.K, p.grid) as mp:
            zs = mp.solve(p.m, p.lam, p.beta, iters, precision=prec, kernel="fused", check_every=e)
            one = mp.stats()
        assert np.array_equal(F.double().cpu().numpy(), zs)
        assert one["hist_iter"] == st["hist_iter"]
        for a, b in (("hist_objective", 1e-12), ("hist_znorm", 1e-12), ("hist_dual", 1e-9)):
            for x, y in zip(st[a], one[a]):
                assert x == pytest.approx(y, rel=b), (p.grid, prec, a)
        ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, iters, track_every=e)
        J = {k: v for (k, v, _) in ref["hist"]}
        say("served monitored", p.grid, prec, iters, e, st["hist_objective"][-1], J[iters])
        for k, v in zip(st["hist_iter"], st["hist_objective"]):
            assert v == pytest.approx(J[k], rel=J_TOL[prec]), (p.grid, prec, k)


def test_served_masked_jobs(torch_cuda, jobs):
    """Masked served jobs (ssmap_server_submit_masked; the maskless footnote of
    Sec. II-C): bitwise the single solve with the same mask (ssmap_set_mask,
    fused kernel), zero outside, within tolerance of the oracle's masked solve,
    and NaN data outside the mask never read; a masked job shares the server
    with an unmasked one and takes monitoring."""
    torch = torch_cuda
    p2 = synth.generate("c1", grid=(29, 23, 1), iters=30)
    yy, xx = np.mgrid[0:23, 0:29]
    m2 = (((xx - 14) ** 2 + (yy - 11) ** 2 < 100) & ~((xx - 16) ** 2 + (yy - 12) ** 2 < 6)).reshape(-1)
    p3 = synth.generate("c2", grid=(19, 11, 5), iters=17)
    zz, yy, xx = np.mgrid[0:5, 0:11, 0:19]
    m3 = ((((xx - 9) / 8.0) ** 2 + ((yy - 5) / 4.5) ** 2 + ((zz - 2) / 2.2) ** 2) < 1.0).reshape(-1)
    cases = [(p2, "fp64", 30, m2, 6), (p3, "fp32", 17, m3, 0), (jobs[0][0], "fp32", 20, None, 0)]
    Ms = []
    for p, prec, _, mask, _ in cases:
        m = p.m.copy()
        if mask is not None:
            m[~mask] = np.nan                          # outside rows are never read
        Ms.append(torch.tensor(m, dtype=getattr(torch, TORCH_T[prec]), device="cuda"))
    torch.cuda.synchronize()
    with _ffi.Server(4e9, 4) as sv:
        ids = []
        for (p, prec, iters, mask, every), M in zip(cases, Ms):
            d = sv.add_dictionary(p.K)
            ids.append(sv.submit(d, p.grid, M, p.lam, p.beta, iters, ready=True, precision=prec,
                                 mask=mask, check_every=every))
        sv.drain()
        infos = [sv.poll(i) for i in ids]
        sts = [sv.job_stats(i) for i in ids]
        Fs = [sv.result(i) for i in ids]
    for (p, prec, iters, mask, every), F, info, st in zip(cases, Fs, infos, sts):
        assert info["status"] == _ffi.SSMAP_OK
        z = F.double().cpu().numpy()
        with _ffi.Mapper(p.K, p.grid) as mp:
            if mask is not None:
                mp.set_mask(mask)
            zs = mp.solve(p.m, p.lam, p.beta, iters, precision=prec, kernel="fused", check_every=every)
            one = mp.stats()
        assert np.array_equal(z, zs), (p.grid, prec)
        assert info["xi_p"] == pytest.approx(one["xi_p"], rel=1e-13)
        ref = oracle.ladmm(p.K, p.m, p.grid, p.lam, p.beta, iters, mask=mask)
        err = np.linalg.norm(z - ref["z"]) / np.linalg.norm(ref["z"])
        say("served masked", p.grid, prec, "inside", None if mask is None else int(mask.sum()), err)
        assert err <= TOL[prec]
        if mask is not None:
            assert np.all(z[~mask] == 0.0)
        if every:
            assert st["hist_iter"] == one["hist_iter"] and len(st["hist_iter"]) > 0
            for x, y in zip(st["hist_objective"], one["hist_objective"]):
                assert x == pytest.approx(y, rel=1e-12)
