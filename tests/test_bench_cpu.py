"""Host-side checks of the benchmark script: it refuses more than one GPU
before touching the GPU, and it names the kernel each recorded launch used
(the roofline's dominant kernel is matched to the profiled one by name)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_names_of_launch_records():
    b = _bench()
    rec = lambda k, q, **f: dict(kind=f.pop("kind", "cluster"), k=k, qubits=q, **f)
    assert b.kernel_name(rec(6, [1, 3, 9, 12, 20, 25], mfma=True)) == "k_cluster_f32_split6<false, false>"
    assert b.kernel_name(rec(6, [0, 3, 9, 12, 20, 25], mfma=True)) == "k_cluster_f32_split6<true, false>"
    assert b.kernel_name(rec(6, [0, 3, 9, 12, 20, 25], mfma=True, stats=True)) == "k_cluster_f32_split6<true, true>"
    assert b.kernel_name(rec(6, [1, 2, 3, 4, 7, 14], mfma=True, staged=True)) == "k_cluster_f32_split6s<false>"
    assert b.kernel_name(rec(6, [0, 1, 2, 3, 21, 22], mfma=True, staged=True)) == "k_cluster_f32_split6s<true>"
    assert b.kernel_name(rec(4, [18, 20, 24, 26], mfma=True, staged=True)) == "k_cluster_f32_stage<4, 6, false>"
    assert b.kernel_name(rec(5, [0, 9, 14, 16, 26], mfma=True)) == "k_cluster_f32_mfma<5, 2, true, false>"
    assert b.kernel_name(rec(5, [1, 9, 14, 16, 26], mfma=True, stats=True)) == "k_cluster_f32_mfma<5, 2, false, true>"
    assert b.kernel_name(rec(3, [2, 5, 9])) == "k_cluster_valu<float, 3>"
    # with the state's size: 2- and 3-qubit clusters on >= k + 6 qubits take the staged form
    assert b.kernel_name(rec(3, [2, 5, 9]), n=34) == "k_cluster_valu_staged<float, 3, false>"
    assert b.kernel_name(rec(2, [2, 5], stats=True), n=34) == "k_cluster_valu_staged<float, 2, true>"
    assert b.kernel_name(rec(3, [2, 5, 6]), n=8) == "k_cluster_valu<float, 3>"
    assert b.kernel_name(rec(2, [2, 9]), dbl=True, n=30) == "k_cluster_valu_staged<double, 2, false>"
    assert b.kernel_name(rec(6, [1, 3, 9, 12, 20, 25], mfma=True), k6_kernel=1) == "k_cluster_f32_gauss6<false>"
    # 6-qubit clusters on the fp32 matrix cores (the real-split kernel, direct only)
    assert b.kernel_name(rec(6, [1, 3, 9, 12, 20, 25], mfma=True), k6_kernel=0) == \
        "k_cluster_f32_mfma<6, 1, false, false>"
    # float64 states
    assert b.kernel_name(rec(5, [1, 9, 14, 16, 26], mfma=True), dbl=True) == "k_cluster_f64_mfma<5, 2, 256>"
    assert b.kernel_name(rec(6, [1, 9, 14, 16, 26, 27], mfma=True), dbl=True) == "k_cluster_f64_mfma<6, 1, 512>"
    assert b.kernel_name(rec(5, [0, 1, 2, 16, 26], mfma=True, staged=True), dbl=True) == \
        "k_cluster_f64_stage<5, 5, 512>"
    assert b.kernel_name(rec(3, [0, 1, 2], mfma=True, staged=True), dbl=True) == "k_cluster_f64_stage<3, 5, 256>"
    pair = rec(5, [0, 1, 2, 3, 4, 5, 6, 7, 8, 9], kind="pair")
    assert b.kernel_name(pair) == "k_cluster_f32_multi<2, 8>"
    assert b.kernel_name(pair, pair_tile=10) == "k_cluster_f32_pair10<12>"


def test_cpu_baseline_runs_the_whole_circuit():
    """The CPU-baseline leg runs the oracle over every gate of the circuit it
    is given (no sampling) and records the host it ran on."""
    import numpy as np

    import oracle
    from supremacy_inputs import supremacy_circuit
    b = _bench()
    circ = supremacy_circuit(3, 4, 12, seed=1)
    kept, dropped = oracle.drop_trailing_diagonal(circ)
    rec, psi = b.cpu_baseline(kept)
    assert rec["kind"] == "oracle" and rec["unit"] == "s" and rec["cores"] >= 1
    assert "%d gates" % len(kept.gates) in rec["sample"]
    assert rec["host"]["cpus_available"] >= 1 and rec["host"]["ram_GiB"] > 0
    np.testing.assert_array_equal(psi, oracle.run(kept))
