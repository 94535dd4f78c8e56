"""Host logic of the benchmark and of the counter summaries (no GPU): the algorithmic byte
counts behind the roofline, the gate on recorded counter traffic, the single-GPU refusal,
and the steady-state averaging of rocprofv3 counter files."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2511_06824_amd import profile_pcg  # noqa: E402


def test_kernel_bytes_of_the_headline_workload():
    # 2048 x 1024 cells, 9 conditions on 5 operators: 8 B per vector operand per
    # condition-DOF, 16 B of face conductances per operator-DOF
    n = 2048 * 1024
    b = bench.kernel_bytes(n, 9, 5)
    assert b["k_pcg_f"] == (7 * 8 * 9 + 16 * 5) * n == 1224736768
    assert b["k_pcg_a"] == (3 * 8 * 9 + 16 * 5) * n == 620756992
    assert b["k_pcg_b"] == (6 * 8 * 9 + 16 * 5) * n == 1073741824
    # the one-launch average is the mean of an odd (8 operands) and an even (6) launch
    odd, even = (8 * 8 * 9 + 80) * n, (6 * 8 * 9 + 80) * n
    assert b["k_pcg_f"] == (odd + even) // 2
    # the strip kernel: r, u_prev read, u, r written (4 operands), p on odd launches (+2)
    assert b["k_pcg_w"] == (5 * 8 * 9 + 16 * 5) * n == 922746880
    assert b["k_pcg_w"] == ((6 * 8 * 9 + 80) * n + (4 * 8 * 9 + 80) * n) // 2


def test_recorded_traffic_needs_the_current_kernel_sources(tmp_path, monkeypatch):
    root = tmp_path / "repo"
    shutil.copytree(os.path.join(ROOT, "paper_2511_06824_amd", "csrc"), root / "paper_2511_06824_amd" / "csrc")
    (root / "profiles").mkdir()
    prof = root / "profiles" / "pcg_joint_textured_2048x1024_traffic.md"
    monkeypatch.setattr(bench, "ROOT", str(root))
    digest = bench.kernel_source_digest()
    prof.write_text(f"kernel source digest: {digest}\ntraffic bytes per launch k_pcg_f: 123456\n")
    assert bench.recorded_traffic("k_pcg_f") == 123456
    assert bench.recorded_traffic("k_pcg_a") is None
    # an edited comment keeps the recorded figure; changed code makes it stale
    src = root / "paper_2511_06824_amd" / "csrc" / "gap_pcg1.hpp"
    src.write_text(src.read_text() + "\n// a comment\n\n")
    assert bench.kernel_source_digest() == digest
    assert bench.recorded_traffic("k_pcg_f") == 123456
    src.write_text(src.read_text() + "constexpr int kProbe = 1;\n")
    assert bench.kernel_source_digest() != digest
    assert bench.recorded_traffic("k_pcg_f") is None
    prof.unlink()
    assert bench.recorded_traffic("k_pcg_f") is None


def test_committed_traffic_summary_matches_the_kernel_sources():
    # the committed counter summary was taken with the kernels in the tree
    for k in ("k_pcg_w", "k_pcg_f", "k_pcg_a", "k_pcg_b"):
        assert bench.recorded_traffic(k) is not None, k


@pytest.mark.parametrize("argv", [["--gpus", "2"], ["--timing-period", "0"]])
def test_bench_refuses_unsupported_runs(argv):
    env = dict(os.environ, WORLD_SIZE="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                       timeout=300, env=env, cwd=ROOT)
    assert r.returncode == 2
    assert r.stdout == ""
    assert r.stderr.strip()


def _counter_csv(path, counter, rows):
    with open(path, "w") as f:
        f.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for did, name, value in rows:
            f.write(f'{did},"{name}","{counter}",{value}\n')


def test_counter_summary_takes_the_steady_state(tmp_path, capsys):
    copy = "__amd_rocclr_copyBuffer"
    kf = "void k_pcg_f<1024, 2, false>(PcgDev const*, int const*, int)"
    ka = "void k_pcg_a<1024, 2>(PcgDev const*, int const*)"
    # a 1 GiB copy read at half rate by FETCH_SIZE; then a solve of the one-launch kernel: a
    # cheap first launch (j = 0), odd / even launches, a closing launch; and one of A
    fetch = [(1, copy, 524288), (2, copy, 524288)]
    write = [(1, copy, 1048576), (2, copy, 1048576)]
    f_vals = [(100, 0), (400, 500), (300, 450), (400, 500), (300, 450), (5, 0)]
    for k, (fv, wv) in enumerate(f_vals):
        fetch.append((10 + k, kf, fv))
        write.append((10 + k, kf, wv))
    for k, (fv, wv) in enumerate([(50, 10), (200, 100), (200, 100), (7, 0)]):
        fetch.append((30 + k, ka, fv))
        write.append((30 + k, ka, wv))
    # the strip kernel: its initial residual (INIT, the fourth argument) is left out, the
    # iteration of the synchronized march (SYNC, the fifth) is summarized
    kwi = "void k_pcg_w<1, -1, 1, true, true>(PcgDev const*, int const*, int)"
    kw = "void k_pcg_w<1, 2, 1, false, true>(PcgDev const*, int const*, int)"
    fetch.append((40, kwi, 999))
    write.append((40, kwi, 999))
    for k, (fv, wv) in enumerate(f_vals):
        fetch.append((50 + k, kw, fv))
        write.append((50 + k, kw, wv))
    fcsv, wcsv = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _counter_csv(fcsv, "FETCH_SIZE", fetch)
    _counter_csv(wcsv, "WRITE_SIZE", write)
    profile_pcg.summarize(str(fcsv), str(wcsv))
    out = capsys.readouterr().out
    assert "scale 2.000" in out and "scale 1.000" in out
    odd = 400 * 1024 * 2 + 500 * 1024
    even = 300 * 1024 * 2 + 450 * 1024
    assert f"| k_pcg_f<1024,2,false>, odd j | 2 | 400.0 | 500.0 | {odd} |" in out
    assert f"| k_pcg_f<1024,2,false>, even j | 2 | 300.0 | 450.0 | {even} |" in out
    assert f"| k_pcg_f<1024,2,false>, average | 4 | | | {(odd + even) // 2} |" in out
    assert f"| k_pcg_a<1024,2> | 2 | 200.0 | 100.0 | {200 * 1024 * 2 + 100 * 1024} |" in out
    assert f"| k_pcg_w<1,2,1,false,true>, odd j | 2 | 400.0 | 500.0 | {odd} |" in out
    assert "k_pcg_w<1,-1,1,true,true>" not in out
