"""Host-side parts of bench.py that run without a GPU: the one-GPU contract, the rule
that stored HBM counters count only for the kernel sources they were taken on, and
the per-level descriptor sizes used for the algorithmic byte counts."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402  (imports no GPU module at the top level)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stored_traffic_follows_the_source_hash(monkeypatch):
    path = os.path.join(ROOT, "profiles", "pmc_3d256.txt")
    recorded = [l.split(":", 1)[1].strip() for l in open(path) if l.startswith("source_hash:")][0]
    monkeypatch.setattr(bench, "source_hash", lambda: recorded)
    v = bench.stored_traffic("3d256", "fwd_mid")
    assert v is not None and 1e8 < v < 2e8          # bytes per dispatch of a 256^3 pass
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)
    assert bench.stored_traffic("3d256", "fwd_mid") is None
    assert bench.stored_traffic("no_such_workload", "fwd_mid") is None


def test_source_hash_is_stable_and_short():
    h = bench.source_hash()
    assert h == bench.source_hash() and len(h) == 16


def test_per_level_sizes_add_up_to_the_descriptor():
    from paper_2103_09686_amd import dmcr
    for shape, C, L, P in [((64, 64, 64), 2, 3, 16), ((512, 512), 1, 3, 64), ((256, 256, 256), 1, 1, 32)]:
        spec = dmcr.make_spec(shape, C, L, P)
        assert sum(bench.K_level(spec, l) for l in range(L)) == dmcr.dmcr_descriptor_size(spec)
