"""Host-side checks of bench.py (no GPU): the one-GPU refusal and the algorithmic bytes that
price the host-driven solvers' roofline."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_host_driven_bytes_per_point_iteration():
    b = _bench()
    # single systems: step with the x and r updates 128 B + r^T z and the p update 64 B
    assert b.host_driven_bytes(False, 0, (24, 24, 24)) == 192.0
    # three fused preconditioner passes on axes <= 32, seven GEMM passes beyond, 32 B each
    assert b.host_driven_bytes(True, 0, (24, 24, 24)) == 192.0 + 3 * 32.0
    assert b.host_driven_bytes(True, 0, (48, 48, 48)) == 192.0 + 7 * 32.0
    # block kernels: q = A p 32 B, alpha step 128 B, beta step 80 B
    assert b.host_driven_bytes(False, 4, (24, 24, 24)) == 240.0
    assert b.host_driven_bytes(True, 2, (24, 24, 24)) == 240.0 + 3 * 32.0
    assert b.ALG_BYTES == {"fp64": 96.0, "mixed": 48.0}
