"""Host-side checks of bench.py that need no GPU: the one-GPU contract and the
roofline bookkeeping (algorithmic contraction flops of the benchmark workload)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_contraction_flops_of_the_benchmark_workload():
    # per (walker, path) and vector: 2 N M^2 (Y = Phi_T^T L_g) + 2 (4 M N^2 + 8 N^2)
    # (Y Theta for both spins, real by complex, and the complex tr(f f)); M = 64, N = 16,
    # 256 vectors, 512 walkers x 8 paths
    import bench
    per_path = bench.contraction_flops(64, 16, 256)
    assert per_path == 256 * (2 * 16 * 64 * 64 + 2 * (4 * 64 * 16 * 16 + 8 * 16 * 16))
    assert abs(per_path * 512 * 8 - 279.2e9) < 0.1e9
