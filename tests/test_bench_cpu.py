"""Host-side checks of bench.py that need no GPU: the one-GPU contract and
the helpers that stamp the JSON line."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_odd_step_count_with_the_two_step_kernel_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "7"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "even" in r.stderr


def test_fp64_arithmetic_mode_is_refused_outside_the_two_phase_legs():
    for leg in ("channel", "d3q19", "phase3d", "adjoint"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--leg", leg,
                            "--prec", "fp32_arith64"], capture_output=True, text=True, timeout=120)
        assert r.returncode == 2
        assert "two-phase" in r.stderr


def test_source_hash_and_host_description():
    sys.path.insert(0, ROOT)
    import bench
    h1, h2 = bench.kernel_source_hash(), bench.kernel_source_hash()
    assert h1 == h2 and len(h1) == 64
    host = bench.host_cpu()
    assert host["nproc"] >= 1
