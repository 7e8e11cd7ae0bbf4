"""Host logic of bench.py (no GPU): the algorithmic byte counts per lattice
update, the source-hash gate on measured traffic, and the refusal of runs
on more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    sys.path.insert(0, ROOT)
    import bench
    return bench


@pytest.fixture(scope="module")
def W():
    from paper_1407_6704_amd import workloads
    return workloads


def test_collide_and_moments_bytes_per_node(B, W):
    # 2 Q populations (read and write) of 4 or 2 bytes plus the D-component force
    cases = [(W.C1, 2 * 9 * 4 + 8), (W.C2, 2 * 19 * 4 + 12), (W.C3, 2 * 19 * 2 + 12),
             (W.C2_D3Q15, 2 * 15 * 4 + 12)]
    for w, per_node in cases:
        assert B.algorithmic_bytes("collide", w, w.n_particles) == w.nodes * per_node
    assert B.algorithmic_bytes("collide", W.C1, 0) == W.C1.nodes * 2 * 9 * 4      # no particles, no force read
    assert B.algorithmic_bytes("moments", W.C2, W.C2.n_particles) == W.C2.nodes * (19 * 4 + 16)
    assert B.algorithmic_bytes("collide", W.C1, W.C1.n_particles) == 335544320


def test_measured_traffic_follows_the_kernel_source(B, monkeypatch):
    # the hash covers the kernel's own function text, the device routines
    # that carry its arithmetic, and the device header
    for k, parts in B.KERNEL_SOURCES.items():
        for src, name in parts:
            txt = B.kernel_text(src, name)
            assert f" {name}(" in txt.splitlines()[0] + txt.splitlines()[1] and txt.endswith("}")
    assert B.source_sha("spread") != B.source_sha("spread_collide")
    sha = B.source_sha("collide")
    assert len(sha) == 16 and sha != B.source_sha("moments")
    rec = {"fetch_bytes": 1.0e9, "write_bytes": 2.0e9, "kernel_sha": sha}
    monkeypatch.setitem(B.MEASURED_TRAFFIC, ("collide", "c2"), rec)
    assert B.measured_traffic("collide", "c2") == 3.0e9
    assert B.measured_traffic("collide", "no_such_workload") is None
    monkeypatch.setattr(B, "source_sha", lambda kernel: "0" * 16)
    assert B.measured_traffic("collide", "c2") is None
    # every stored record carries the hash it was measured under
    for rec in B.MEASURED_TRAFFIC.values():
        assert set(rec) == {"fetch_bytes", "write_bytes", "kernel_sha"}


def test_headline_is_the_largest_single_gpu_workload(B, W):
    import argparse  # noqa: F401
    big = max((w for w in (W.C0, W.C1, W.C2, W.C4)), key=lambda w: w.nodes)
    assert big is W.C2
    assert B.workload_name(W.C2) == "c2: D3Q19 256x256x256"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
