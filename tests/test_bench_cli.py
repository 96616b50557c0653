"""The benchmark's command line without a GPU: the one-GPU contract and the
section names it accepts."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=env)


def test_more_than_one_gpu_exits_with_a_message():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_world_size_above_one_exits_too():
    env = dict(os.environ, WORLD_SIZE="2")
    r = run(env=env)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_sections_are_documented():
    import bench  # the repository root is on sys.path (conftest)

    r = run("--help")
    assert r.returncode == 0
    text = "".join(r.stdout.split())   # argparse wraps the list at any character
    for name in bench.SECTIONS + ("ntt_lengths",):
        assert name in text, name
