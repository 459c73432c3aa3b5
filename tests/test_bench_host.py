"""Host logic of bench.py (CPU only): the serving leg's child process is
reported, not fatal, when it fails, and gets the run's options; the flop
count per evaluation."""

import json
import subprocess
import sys
import types

import pytest

import bench


def _args(**kw):
    base = dict(serving_requests=4, serving_max_steps=10, serving_pool_gib=0.01, serving_slots=2, serving_warmup=0)
    base.update(kw)
    return types.SimpleNamespace(**base)


def test_serving_child_result_is_parsed_and_passes_its_options(monkeypatch):
    seen = {}

    def fake_run(cmd, stdout, text, timeout):
        seen["cmd"] = cmd
        line = json.dumps({"requests": 4, "done": 4, "p50_time_to_target_s": None})
        return types.SimpleNamespace(returncode=0, stdout="progress\n" + line + "\n")

    monkeypatch.setattr(subprocess, "run", fake_run)
    out = bench.serving_in_child(_args(serving_warmup=2), 2.6)
    assert out == {"requests": 4, "done": 4, "p50_time_to_target_s": None}
    cmd = seen["cmd"]
    assert cmd[0] == sys.executable and "--serving-child" in cmd
    assert cmd[cmd.index("--serving-target-factor") + 1] == "2.6"
    assert cmd[cmd.index("--serving-warmup") + 1] == "2"


@pytest.mark.parametrize("rc,stdout", [(139, ""), (0, "no json here\n"), (-6, '{"partial": 1}\n')])
def test_serving_child_failure_is_reported(monkeypatch, rc, stdout):
    monkeypatch.setattr(subprocess, "run", lambda *a, **k: types.SimpleNamespace(returncode=rc, stdout=stdout))
    out = bench.serving_in_child(_args(), 1.1)
    assert out["requests"] == 4 and f"status {rc}" in out["error"]


def test_serving_child_timeout_is_reported(monkeypatch):
    def fake_run(cmd, stdout, text, timeout):
        raise subprocess.TimeoutExpired(cmd, timeout)

    monkeypatch.setattr(subprocess, "run", fake_run)
    out = bench.serving_in_child(_args(), 1.1)
    assert "did not finish" in out["error"]


def test_flops_per_eval_is_the_upper_triangle_count():
    # 8 d flops per pair (Re and Im of a complex inner product), N (N - 1) / 2 pairs
    assert bench.flops_per_eval(4096, 64) == 8 * 64 * 4096 * 4095 / 2
    assert bench.flops_per_eval(2, 1) == 8

