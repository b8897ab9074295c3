"""CPU checks of bench.py's own logic: the one-GPU contract, the algorithmic
byte counts the roofline divides by, and that the committed HBM counter
record still belongs to the solver sources (else `traffic` is reported as
null)."""
import json

import pytest
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout == ""


def test_algorithmic_bytes_of_the_dense_update():
    # (2 m n + 2 p q + 2 q n + m + n + p) * 8 on the 2000x500 / 500x2000 workload.
    assert bench.algorithmic_bytes_per_update(2000, 500, 500, 2000, 8) == 84_036_000
    # Brute-force count of the same terms on a small shape.
    m, p, q, n = 7, 3, 4, 5
    terms = [m * n, m * n, p * q, p * q, q * n, q * n, m, n, p]
    assert bench.algorithmic_bytes_per_update(m, p, q, n, 4) == 4 * sum(terms)


def test_algorithmic_bytes_of_the_sparse_update():
    # 512 x 512 blur: 9 nonzeros per row of A and per row / column of B, 17
    # per column of A A^T.
    assert bench.sparse_update_bytes(512, 512, 512, 512, 9, 9, 9, 17) == 364_544
    # R_{i_k} read, ELL index + value of B's rows and columns, X rows read and
    # written plus X_ref read, R rows read and written.
    m, p, q, n, ka, kb, kbt, kg = 10, 6, 4, 8, 2, 3, 2, 5
    want = 8 * n + 12 * (q * kb + n * kbt) + 8 * 3 * ka * q + 8 * 2 * kg * n
    assert bench.sparse_update_bytes(m, p, q, n, ka, kb, kbt, kg) == want


def test_counter_record_matches_the_solver_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles",
                                      "solve_kernel_large_grbk_fp64_counters.json")))
    if rec["source_sha256"] != bench.kernel_source_digest():
        # Counters taken on other sources give no traffic figure at all.
        assert bench.measured_traffic(rec["team_wgs"], rec["updates_per_launch"]) is None
        pytest.skip("the counter record predates the current solver sources")
    traffic = bench.measured_traffic(rec["team_wgs"], rec["updates_per_launch"])
    assert traffic is not None and traffic > 0
    # A different launch (team or length) gets no traffic figure.
    assert bench.measured_traffic(rec["team_wgs"] + 1, rec["updates_per_launch"]) is None
