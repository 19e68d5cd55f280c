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


def test_action_traffic_assigns_exact_counters_to_their_actions(tmp_path, capsys):
    """Per-dispatch counter files whose values are exactly the algorithmic
    bytes of a known launch sequence (FETCH_SIZE in KiB at half the bytes
    read, WRITE_SIZE in KiB at the bytes written, as the copy calibration
    reads them) are assigned action by action, with ratio 1 everywhere."""
    n, w, k = 255 ** 3, 8, 40
    rw = {"A": (48, 32), "A0": (16, 32), "B": (24, 8), "RES": (48, 8), "CDOT": (328, 0), "APPLYW": (360, 16),
          "APPLY": (16, 16), "FIN": (40, 8), "NONE/REDUCE": (0, 0)}
    seq = ["A0", "B"] + ["A", "B"] * 5 + ["RES", "CDOT", "NONE/REDUCE", "APPLYW", "APPLY", "FIN"]
    name = "void tgdk::k_step<tgdk::Tile<3, 4, 4>, 3, false, double>(tgdk::DevProb const*, int const*, int)"
    for which, col, scale in (("fetch", 0, 2.0), ("write", 1, 1.0)):
        lines = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
        lines.append('1,"void tgdk::k_apply<x>(int)",X,123')  # another kernel: ignored
        for i, a in enumerate(seq):
            lines.append(f'{i + 2},"{name}",{which.upper()}_SIZE,{rw[a][col] * n / 1024 / scale}')
        (tmp_path / f"{which}.csv").write_text("\n".join(lines) + "\n")
    bench.action_traffic(str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv"))
    out = capsys.readouterr().out
    rows = {r.split("|")[1].strip(): r.split("|") for r in out.splitlines()[2:]}
    for a in set(seq):
        assert int(rows[a][2]) == seq.count(a), a
        if a != "NONE/REDUCE":
            assert rows[a][5].strip() == "1.000", (a, rows[a])
