"""The seeded workload generators: determinism and the shapes the workloads
promise (sizes, row-length statistics).  Statistics are computed by the CPU
oracle."""
import json
import os

import numpy as np
import pytest

import gen
import oracle


def test_generators_are_deterministic():
    a = gen.lognormal_matrix(5000, 16.0, 1.2, 9)
    b = gen.lognormal_matrix(5000, 16.0, 1.2, 9)
    assert np.array_equal(a.irp, b.irp) and np.array_equal(a.icol, b.icol)
    assert np.array_equal(a.val.view(np.uint64), b.val.view(np.uint64))
    c = gen.lognormal_matrix(5000, 16.0, 1.2, 10)
    assert not np.array_equal(a.icol[:100], c.icol[:100])
    assert np.array_equal(gen.x_uniform(100, 3), gen.x_uniform(100, 3))


def test_random_rows_are_sorted_distinct_and_in_range():
    m = gen.lognormal_matrix(20000, 16.0, 1.2, 4)
    assert oracle.validate_crs(m.n, m.irp, m.icol) == 0
    for i in range(0, m.n, 97):
        r = m.icol[m.irp[i]:m.irp[i + 1]]
        assert np.all(np.diff(r) > 0)


def test_laplace_shape():
    m = gen.laplace_64x64()
    assert (m.n, m.nnz) == (4096, 20224)
    assert set(np.unique(m.val)) == {4.0, -1.0}


@pytest.mark.slow
def test_stencil27_values():
    m = gen.stencil27(16, 16, 16, gen.seed_for(2))
    rows = np.repeat(np.arange(m.n), np.diff(m.irp))
    diag = m.icol == rows
    assert np.all((m.val[diag] >= 26) & (m.val[diag] < 27))
    assert np.all((m.val[~diag] >= -1.1) & (m.val[~diag] < -0.9))


def test_dsweep_table_reproduces_targets():
    tab = gen.dsweep_table()
    assert len(tab["s"]) == 33
    for idx in (0, 1, 8, 16, 24, 32):
        lens = gen.dsweep_lengths(tab["s"][idx])
        irp = np.zeros(lens.shape[0] + 1, np.int64)
        irp[1:] = np.cumsum(lens)
        d = oracle.dmat(lens.shape[0], irp.astype(np.int32))
        assert abs(d - gen.DSWEEP_TARGETS[idx]) <= 0.01
        assert lens.min() >= 1 and lens.max() <= 8192


def test_powerlaw_lengths():
    lens = gen.lognormal_lengths(gen.POWERLAW_N, 16.0, 1.2, 1, 8192, gen.seed_for(3))
    irp = np.zeros(lens.shape[0] + 1, np.int64)
    irp[1:] = np.cumsum(lens)
    d = oracle.dmat(lens.shape[0], irp.astype(np.int32))
    # lognormal with sigma_log = 1.2: D = sqrt(exp(1.44) - 1) = 1.795 before rounding/clipping
    assert abs(d - 1.795) < 0.02
    assert abs(lens.mean() - 16.0) < 0.1


def test_serving_stream_shape():
    jobs = gen.serving_jobs(2048)
    assert len(jobs) == 2048
    assert all(1000 <= j.n <= 500000 for j in jobs)
    assert all(1 <= j.k <= 500 for j in jobs)
    assert [j.kind for j in jobs[:4]] == ["banded", "random", "banded", "random"]
    t = [j.arrival_s for j in jobs]
    assert all(b >= a for a, b in zip(t, t[1:]))
