"""The persistent workers' synchronisation protocol on the CPU: a host-thread model
(tests/cpu_model/grid_protocol.cpp) of the two-level grid barrier, the flat variant
and the control/compute batch hand-off, built with ThreadSanitizer and run with
random interleavings. The model must pass (no race, no early exit from a barrier,
every batch's own descriptor seen once, in order) and must catch two planted
mistakes."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_model", "grid_protocol.cpp")


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("model") / "grid_protocol")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread", SRC, "-o", exe], check=True)
    return exe


def _run(exe, n, rounds, seed, mode, deadline=60):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    return subprocess.run([exe, str(n), str(rounds), str(seed), mode, str(deadline)], capture_output=True, text=True,
                          timeout=deadline + 60, env=env)


@pytest.mark.parametrize("mode", ["two-level", "flat", "handoff"])
@pytest.mark.parametrize("n", [5, 13, 33])
def test_protocol_holds(model, mode, n):
    r = _run(model, n, 200, 1000 + n, mode)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr


@pytest.mark.parametrize("mode,expect", [("two-level-late-gen", "barrier"), ("handoff-same-slot", "descriptor")])
def test_planted_mistakes_are_caught(model, mode, expect):
    # the mistakes show only under some interleavings: a few seeds, all must not pass
    runs = [_run(model, 17, 2000, seed, mode, deadline=2) for seed in (1, 2, 3, 4)]
    caught = [r for r in runs if r.returncode != 0 and expect in r.stderr]
    assert caught, [r.stdout + r.stderr for r in runs]
