"""Host logic of the benchmark (no GPU): the algorithmic bytes per grid
point that the roofline charges to each step-kernel action, counted here
independently as whole vectors read and written, the rule that takes HBM
traffic from the committed counter summary only for the same kernel sources
and launch mix, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _vectors(reads, writes, word):
    return (reads + writes) * word


@pytest.mark.parametrize("w", [8, 4])
def test_phase_bytes_are_whole_vector_passes(w):
    """Phase A reads r_(i-1), t, p, v, e, r^ and writes r_i, e, p, v; phase B
    reads r_i, v, r^ and writes t; the first phase A reads r and r^ and
    writes p, v, e and r_i -- each entry one inner word."""
    b = bench.act_bytes(3, w, 8, 40, False)
    assert b["A"] == _vectors(6, 4, w)
    assert b["B"] == _vectors(3, 1, w)
    assert b["A0"] == _vectors(2, 4, w)
    assert b["NONE"] == 0 and b["REDUCE"] == 0


def test_3d_boundary_bytes_with_a_float64_basis():
    """k = 40 columns of V in float64: c = V^T r reads r and V; w = V d and
    the pending x update read x, e, p, r_i, v_i and V and write x and w; the
    true residual reads x, b and the update and writes r (V read by CDOT,
    not here)."""
    k = 40
    b = bench.act_bytes(3, 8, 8, k, False)
    assert b["CDOT"] == 8 + 8 * k
    assert b["APPLYW"] == 8 + 4 * 8 + 8 * k + 8 + 8
    assert b["RES"] == 8 + 8 + 4 * 8 + 8
    assert b["APPLY"] == 8 + 8 + 8 + 8  # reads w, r; writes r, r^


def test_3d_residual_with_a_float32_basis_reads_v():
    """With V stored in float32 the true residual's pass also forms c, so it
    reads the k float32 columns."""
    k = 40
    assert bench.act_bytes(3, 4, 4, k, True)["RES"] == 8 + 8 + 4 * 4 + 8 + 4 * k


def test_2d_boundary_reads_v_in_the_residual_and_the_apply():
    k = 31
    b = bench.act_bytes(2, 8, 8, k, False)
    assert b["RES"] == 8 + 8 + 4 * 8 + 8 * k + 8
    assert b["APPLY"] == 8 + 8 + 4 * 8 + 8 * k + 8 + 8 + 8


def test_no_deflation_residual_writes_the_inner_residual():
    b = bench.act_bytes(3, 4, 8, 0, True)
    assert b["RES"] == 8 + 8 + 4 * 4 + 8 + 4 + 4  # r^ and the separate float32 r_in


def test_counter_traffic_only_for_the_same_sources_and_launch_mix():
    name = "k_step_f64_255cube_counters.txt"
    kv = {}
    for line in open(os.path.join(ROOT, "profiles", name)):
        if ":" in line and not line.startswith((" ", "#", "`", "|")):
            key, v = line.split(":", 1)
            kv[key.strip()] = v.strip()
    alg = float(kv["algorithmic_bytes_per_launch"].split()[0])
    same_sources = kv["kernel_source_hash"] == bench.kernel_hash()
    got = bench.traffic_from_profiles(name, alg)
    assert got == (float(kv["hbm_bytes_per_launch"]) if same_sources else None)
    assert bench.traffic_from_profiles(name, alg * 1.02) is None
    assert bench.traffic_from_profiles(name, alg * 0.98) is None
    assert bench.traffic_from_profiles("no_such_summary.txt", alg) is None


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env={**os.environ, "HIP_VISIBLE_DEVICES": ""})
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
