"""Host-side behaviour of bench.py that needs no GPU: the one-GPU contract and its CLI."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_unknown_workload_is_rejected():
    r = _bench("--workload", "c9")
    assert r.returncode != 0
    assert "invalid choice" in r.stderr


def _bench_module():
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        sys.path.remove(ROOT)
    return bench


def test_stored_sweep_traffic_matches_the_current_kernel_sources():
    """The HBM traffic figures bench.py reports were measured on the current sources of the
    sweep GEMM, its launches and the block-height table; a change to them must come with new
    counter runs (or bench.py would report no traffic)."""
    bench = _bench_module()
    h = bench.kernel_sources_hash()
    assert bench.SWEEP_TRAFFIC
    for key, tr in bench.SWEEP_TRAFFIC.items():
        assert tr["sources"] == h, key
        assert tr["bytes_per_launch"] > 0


def test_cpu_baseline_terms_scale_by_their_own_exponents():
    """The oracle cost model: LU grows as n^3, a solve pair as n^2 m0, Rayleigh-Ritz by its
    fitted n^2 m0, n m0^2 and m0^3 terms; nodes run in parallel over the threads."""
    bench = _bench_module()
    cm = {"t_lu": 2.0, "ns": 1024, "t_solve": 0.5, "ms": 256, "rr_coef": (1e-9, 2e-9, 3e-9)}
    a = bench.oracle_estimate(cm, 1024, 256, 8, 3, 4, 8)
    b = bench.oracle_estimate(cm, 2048, 512, 8, 3, 4, 8)
    assert abs(b["terms_s"]["lu_per_node"] / a["terms_s"]["lu_per_node"] - 8.0) < 1e-12
    s_a = a["terms_s"]["solve_pair_per_node_per_filter"]
    s_b = b["terms_s"]["solve_pair_per_node_per_filter"]
    assert abs(s_b / s_a - 8.0) < 1e-12  # (2n)^2 (2 m0) / (n^2 m0)
    rr = 1e-9 * 1024 ** 2 * 256 + 2e-9 * 1024 * 256 ** 2 + 3e-9 * 256 ** 3
    assert abs(a["terms_s"]["rayleigh_ritz_per_iteration"] - rr) < 1e-9 * rr
    per_node = 2.0 + 4 * 0.5
    assert abs(a["single_thread_s"] - (8 * per_node + 3 * rr)) < 1e-9 * a["single_thread_s"]
    assert abs(a["node_parallel_s"] - (per_node + 3 * rr)) < 1e-9 * a["node_parallel_s"]
    c = bench.oracle_estimate(cm, 1024, 256, 8, 3, 4, 3)  # 8 nodes on 3 threads: 3 rounds
    assert abs(c["node_parallel_s"] - (3 * per_node + 3 * rr)) < 1e-9 * c["node_parallel_s"]
