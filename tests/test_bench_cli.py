"""bench.py's command line on the host: one GPU only, and the documented flags."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_help_lists_the_legs():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--fp64-steps", "--free-steps", "--report-steps", "--compare-steps",
                 "--ensemble", "--hw-queues", "--study", "--reports-jsonl", "--windows-json", "cscan", "nonorth", "scf"):
        assert flag in r.stdout


def test_step_reports_are_written_one_json_object_per_line(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    from paper_2303_00689_amd import binding
    path = tmp_path / "reports.jsonl"
    log = bench.ReportLog(str(path), binding, "c840")
    fields = {"E_tot": -1.5, "KE": 0.25, "U": -1.75, "TS": 0.01, "T_ion": 300.0, "mu": -4.2, "W0": 1e-3,
              "relres": 0.1, "rank": 6, "levels": 9, "mu_passes": 0}
    log.write("free_trajectory", "dm64_bf16x3", 1, dict(fields, status=0))
    log.write("split", "dm64_bf16x3", 2, dict(fields, status=-7))
    log.close()
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert [r["step"] for r in lines] == [1, 2]
    assert lines[0]["status"] == binding.STATUS[0] and lines[1]["status"] == binding.STATUS[-7]
    assert lines[1]["leg"] == "split" and lines[1]["workload"] == "c840"
    for k, v in fields.items():
        assert lines[0][k] == v
    # no path: nothing is written
    quiet = bench.ReportLog("", binding, "c840")
    quiet.write("free_trajectory", "fp64", 1, dict(fields, status=0))
    quiet.close()
