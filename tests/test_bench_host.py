"""Host logic of bench.py that runs without a GPU: the one-GPU refusal, the guard that
attaches counter-measured DRAM bytes to a roofline only when they were taken on the current
fine-sweep sources at the same Newton tolerance and adaptive setting, and the extrapolation
of the CPU oracle's sample to whole steady states."""
import hashlib
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def _summary(tmp_path, sha, tol_newton="1e-10", tol_adapt=None):
    text = [f"fine-sweep sources sha1 (fine_chain.hpp + fine.hip): {sha}", f"tol_newton: {tol_newton}"]
    if tol_adapt is not None:
        text.append(f"tol_adapt: {tol_adapt}")
    text += ["traffic_bytes_per_launch: 6000", "algorithmic_bytes_per_launch: 90000", "launch_ms: 30.5"]
    p = tmp_path / "counters.md"
    p.write_text("\n".join(text) + "\n")
    return str(p)


def _current_sha():
    return hashlib.sha1(b"".join(open(f, "rb").read() for f in bench.FINE_SRC)).hexdigest()


def test_counter_summary_taken_on_the_current_sources_is_used(tmp_path):
    p = _summary(tmp_path, _current_sha(), tol_adapt="0.001")
    t = bench.measured_traffic(1e-10, p, 1e-3)
    assert t == {"bytes": 6000, "algorithmic_bytes_same_launch": 90000, "launch_ms": 30.5}


@pytest.mark.parametrize("case", ["other sources", "other newton tolerance", "other adaptive setting",
                                  "adaptive line missing"])
def test_counter_summary_of_other_launches_is_not_used(tmp_path, case):
    sha, tn, ta, want_ta = _current_sha(), "1e-10", "0.001", 1e-3
    if case == "other sources":
        sha = "0" * 40
    elif case == "other newton tolerance":
        tn = "1e-13"
    elif case == "other adaptive setting":
        want_ta = 0.0
    else:
        ta = None                      # a summary without the line was taken at fixed tolerance
    p = _summary(tmp_path, sha, tn, ta)
    assert bench.measured_traffic(1e-10, p, want_ta) is None


def test_summary_without_adaptive_line_serves_fixed_tolerance_runs(tmp_path):
    p = _summary(tmp_path, _current_sha())
    assert bench.measured_traffic(1e-10, p, 0.0) is not None


def test_cpu_extrapolation_counts_the_gpu_solves_sweeps_and_corrections():
    prob = SimpleNamespace(N=40, m=50)
    smp = {"t_sweep": 4.0, "t_coarse": 0.5, "t_step_seq": 0.01, "cores": 16, "tol_newton": 1e-10,
           "seq_steps": 100, "host": {"nproc": 16}}
    # 14 iterations: 15 sweeps and 14 corrections; nested start of 8 iterations at 2 steps per
    # chain: 9 sweeps at 2/50 of the cost and 8 corrections; route S: 3 periods of 2,000 steps
    out = bench.cpu_extrapolate(prob, smp, 14, 8, 2, 3)
    t_p = 15 * 4.0 + 14 * 0.5 + 9 * 4.0 * 2 / 50 + 8 * 0.5
    assert out["value"] == pytest.approx(1.0 / t_p)
    assert out["route_s"]["value"] == pytest.approx(1.0 / (3 * 40 * 50 * 0.01))
    assert out["cores"] == 16 and out["kind"] == "oracle"
