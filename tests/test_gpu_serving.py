"""The continuous-batching server on the GPU.

Each job's y_k must be bitwise identical when the job runs alone and when it
runs in the mix (the server only uses deterministic formats), and must agree
with the CPU oracle's binary64 chain on the same binary32 inputs within the
binary32 bound of the chain."""
import math

import numpy as np
import pytest

import gen
import oracle
from _gpu import lib_ready

pytestmark = pytest.mark.gpu


def small_specs(count, n_max=20000):
    return gen.serving_jobs(count, rate_per_s=0.0, n_max=n_max)


def oracle_chain(job):
    """y_k of the job's chain, in binary64 from the stored binary32 data."""
    irp = job.irp.numpy()
    icol = job.icol.numpy()
    val = job.val.numpy().astype(np.float64)
    x = job.x0.numpy().astype(np.float64)
    for t in range(job.k):
        y = oracle.spmv_crs(job.n, irp, icol, val, x)
        x = y * 2.0 ** (-job.shift)
    return y


def test_alone_equals_mix_and_matches_oracle():
    spmvat = lib_ready()
    from paper_2407_00019_amd import serve
    specs = small_specs(24)
    for s in specs:
        s.k = min(s.k, 6)
    jobs = serve.build_jobs(specs)
    table = serve.load_table()
    for policy in (0, 1):
        res, _ = serve.run(jobs, policy, slots=6, hbm_cap=2 << 30, table=table, arrivals=[0.0] * len(jobs))
        assert len(res) == len(jobs) and all(r.status == 0 for r in res)
        mixed = {j.id: j.y.numpy().copy() for j in jobs}
        fmt_mix = {r.id: r.format for r in res}
        for j in jobs:
            r1, _ = serve.run([j], policy, slots=1, hbm_cap=2 << 30, table=table, arrivals=[0.0])
            assert r1[0].status == 0
            assert r1[0].format == fmt_mix[j.id]
            assert np.array_equal(j.y.numpy().view(np.uint32), mixed[j.id].view(np.uint32)), (policy, j.id)
            yref = oracle_chain(j)
            # each step is a binary32 dot product (bound gamma_(l+1)); k steps compound
            lmax = int(np.diff(j.irp.numpy()).max())
            u = 2.0 ** -24
            tol = j.k * (lmax + 1) * u / (1 - (lmax + 1) * u) * 4
            err = np.linalg.norm(j.y.numpy() - yref) / max(np.linalg.norm(yref), 1e-300)
            assert err <= max(tol, 1e-6), (policy, j.id, err, tol)


def test_admission_respects_the_memory_cap():
    lib_ready()
    from paper_2407_00019_amd import serve
    specs = small_specs(16, n_max=50000)
    jobs = serve.build_jobs(specs)
    cap = 64 << 20
    res, _ = serve.run(jobs, 0, slots=8, hbm_cap=cap, arrivals=[0.0] * len(jobs))
    assert len(res) == len(jobs)
    assert all(r.status == 0 for r in res)
    assert all(r.device_bytes <= cap for r in res)


def test_too_large_job_is_reported_not_run():
    lib_ready()
    from paper_2407_00019_amd import serve
    jobs = serve.build_jobs(small_specs(2, n_max=5000))
    res, _ = serve.run(jobs, 1, slots=2, hbm_cap=8192, arrivals=[0.0, 0.0])
    assert sorted(r.status for r in res) == [3, 3]
