"""Host-side checks of bench.py that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    msg = r.stdout + r.stderr
    assert "one GPU" in msg and "--gpus 2" in msg
    assert not r.stdout.lstrip().startswith("{")   # no benchmark line


def test_kernel_source_hash_is_stable_and_covers_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 16
    for src in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, src)), src


def test_executed_share_counts_three_product_launches_at_three_quarters():
    # a GPE step runs mode 1 with the prologue phase (tune key load path
    # 0 + 8, else 0) and modes 2, 3 on strided fibres (load path 1)
    sys.path.insert(0, ROOT)
    import bench
    t = lambda load, cls: {"load": load, "rows": 512, "fibres": 65536, "class": cls, "us": 1.0}
    assert bench.executed_share([]) == 1.0
    assert bench.executed_share([t(0, 3), t(1, 3), t(8, 3), t(9, 3)]) == 1.0
    assert abs(bench.executed_share([t(0, 3), t(1, 4), t(8, 8)]) - (0.75 + 2) / 3) < 1e-15
    assert abs(bench.executed_share([t(0, 8), t(1, 9)]) - 0.75) < 1e-15   # no key with the phase
    assert abs(bench.executed_share([t(0, 8), t(1, 4), t(8, 3)]) - 1.0) < 1e-15
