"""Host-side checks of bench.py (no GPU): the one-GPU refusal, the algorithmic bytes that
price the host-driven solvers' roofline, the subspace-convergence report and the kernel a
cycle step runs."""
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


def test_subspace_convergence_report():
    b = _bench()
    # a fixed count has no energy test
    assert b.subspace_converged([[3, 3]], 0.0, 3) is None
    assert b.ec_label([[3, 3]], 0.0, 3) == "fixed count of 3 subspace iterations per frequency"
    # with the test, a frequency that used the whole cap did not converge
    assert b.subspace_converged([[50, 12, 50], [7]], 1e-8, 50) == [[False, True, False], [True]]
    assert b.ec_label([[50, 12, 50], [7]], 1e-8, 50).startswith(
        "not converged: 2 of 4 frequencies stopped at the cap of 50")
    assert b.ec_label([[12, 9]], 1e-8, 50) == "energy test (ec_tol 1e-08) held at every frequency"


def test_cycle_steps_below_mixed_min_omega_run_the_fp64_kernel():
    b = _bench()
    assert b.cycle_kernel_class(0.311, "mixed", 0.2) == "mixed"
    assert b.cycle_kernel_class(0.2, "mixed", 0.2) == "mixed"
    assert b.cycle_kernel_class(0.1132, "mixed", 0.2) == "fp64"
    assert b.cycle_kernel_class(0.0203, "fp64", 0.0) == "fp64"
