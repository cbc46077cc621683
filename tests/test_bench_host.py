"""Host logic of bench.py, on the CPU: the one-GPU contract, the pass
accounting behind `roofline`, and the check that ties the counter summary to
the kernel sources it was taken on."""
import json
import os
import subprocess
import sys

import pytest

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_pass_accounting_two_steps_per_pass():
    """Two steps per pass move the state once: hbm_frac follows the pass's
    own bytes, the one-step figures are named as equivalents."""
    nodes = 256 ** 3
    res = {"ms_per_step": 0.3, "steps_per_pass": 2, "pass_bytes": 2 * 19 * 4 * nodes,
           "bytes_per_node": 152.0}
    bench.pass_accounting(res, nodes)
    assert res["pass_ms"] == pytest.approx(0.6)
    assert res["pass_gbs"] == pytest.approx(2 * 19 * 4 * nodes / 0.6e-3 / 1e9)
    assert res["hbm_frac"] == pytest.approx(res["pass_gbs"] / 8000.0)
    assert res["one_step_equiv_gbs"] == pytest.approx(2 * res["pass_gbs"])
    assert res["mlups_over_one_step_roofline"] == pytest.approx(
        nodes / 0.3e-3 / (8000e9 / 152.0))


def test_pass_accounting_one_step_per_pass_equals_equivalent():
    nodes = 1000
    res = {"ms_per_step": 1.0, "steps_per_pass": 1, "pass_bytes": 152.0 * nodes,
           "bytes_per_node": 152.0}
    bench.pass_accounting(res, nodes)
    assert res["pass_gbs"] == pytest.approx(res["one_step_equiv_gbs"])


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    a = tmp_path / "a.hpp"
    a.write_text("int f(int x) { return x + 1; } // one\n/* block */\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["a.hpp"])
    h0 = bench.kernel_source_hash()
    a.write_text("// new comment\nint f(int x)   {\n  return x + 1;\n}\n")
    assert bench.kernel_source_hash() == h0
    a.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash() != h0


def test_traffic_is_null_once_the_kernel_changed(tmp_path, monkeypatch):
    prof = tmp_path / "traffic.json"
    prof.write_text(json.dumps({"kernel_source_hash": "0" * 16, "bytes_per_launch": 1.0}))
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(prof))
    value, note = bench.traffic_from_profile()
    assert value is None and "changed" in note
    prof.write_text(json.dumps({"kernel_source_hash": bench.kernel_source_hash(),
                                "bytes_per_launch": 2.5e9}))
    assert bench.traffic_from_profile()[0] == 2.5e9


def test_committed_traffic_summary_is_plausible():
    """The committed counter summary of the headline kernel: reads and
    writes of at least the algorithmic bytes and at most a tenth more."""
    with open(bench.PROFILE_TRAFFIC) as fh:
        prof = json.load(fh)
    alg = 2 * 19 * 4 * 256 ** 3
    assert prof["algorithmic_bytes_per_launch"] == alg
    assert 1.0 <= prof["bytes_per_launch"] / alg <= 1.1
    assert prof["write_bytes_per_launch"] == pytest.approx(alg / 2, rel=1e-4)
