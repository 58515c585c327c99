"""Host logic of the benchmark's reporting: the counter-measured traffic of a sweep is reported
only while the sources it was measured on are unchanged (else null), never for a kernel that was
not measured; the algorithmic bytes of a sweep are the field read and written once plus one read
of each optic map."""

import hashlib
import os

import bench


def _digest(rel):
    with open(os.path.join(bench.ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def test_traffic_follows_the_sources_it_was_measured_on(monkeypatch):
    kernel = "col_sweep_adj"
    rel = next(iter(bench.TRAFFIC_SOURCES[kernel]))
    fetch, write = bench.MEASURED_TRAFFIC[kernel]
    # digests of the sources as they are: the stored figure
    monkeypatch.setitem(bench.TRAFFIC_SOURCES, kernel, {rel: _digest(rel)})
    assert bench.measured_traffic(kernel) == fetch + write
    # a source changed since the counters were taken: unknown
    monkeypatch.setitem(bench.TRAFFIC_SOURCES, kernel, {rel: "0" * 64})
    assert bench.measured_traffic(kernel) is None
    # a source that is missing: unknown
    monkeypatch.setitem(bench.TRAFFIC_SOURCES, kernel, {"no/such/file.hip": _digest(rel)})
    assert bench.measured_traffic(kernel) is None


def test_unmeasured_kernel_has_no_traffic():
    assert bench.measured_traffic("exact_cols") is None
    assert bench.measured_traffic("no_such_kernel") is None


def test_every_measured_kernel_names_its_sources():
    for kernel in bench.MEASURED_TRAFFIC:
        srcs = bench.TRAFFIC_SOURCES[kernel]
        assert srcs and all(len(d) == 64 for d in srcs.values())
        assert all(os.path.exists(os.path.join(bench.ROOT, rel)) for rel in srcs)


def test_sweep_bytes():
    n = 4096
    assert bench.sweep_bytes(n, 0) == 2 * n * n * 8
    assert bench.sweep_bytes(n, 2) == 2 * n * n * 8 + 2 * n * n * 4
